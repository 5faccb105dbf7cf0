"""CPU checks of the C ABI: the library loads and exports every function the
public header declares, and the binding names them all.  No GPU call is made."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "fqnm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fqnm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for core in ("fqnm_create", "fqnm_step", "fqnm_reconstruct", "fqnm_destroy",
                 "fqnm_batch_run", "fqnm_server_submit", "fqnm_server_poll"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2604_06947_amd import fqnm as F
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("libfqnm.so not built")
    L = F.lib()
    for name in declared():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2604_06947_amd import fqnm as F
    assert sorted(F.EXPORTED) == declared()
    for name in declared():
        assert callable(getattr(F, name)), name


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2604_06947_amd import fqnm as F
    monkeypatch.setattr(F, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(F, "_lib", None)
    with pytest.raises(ImportError):
        F.lib()
