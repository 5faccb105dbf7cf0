"""fqnm_invariants_get_noalloc (the variant for callers that cannot allocate)
against fqnm_invariants_get, through the C ABI: on a large state whose blocks
reduce more than the minimum cell count, then on a smaller one, so the second
call reuses the shared static scratch after a larger call; also on int64,
outflow (ledger) and Euler contexts."""
import numpy as np
import pytest

from paper_2604_06947_amd import fqnm as F
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctx_scalar(n, itype, bc, steps, seed):
    q0 = W.random_states(n, -30000, 30000, seed=seed)
    q0 = q0.astype(np.int32 if itype == F.I32 else np.int64)
    prob = F.make_problem(F.FLUX_UPWIND, 1e-4, 0.5, n, itype=itype, bc=bc, a=1.0)
    h = F.fqnm_create(prob, q0)
    F.fqnm_step(h, steps)
    return h


def _same(h):
    a = F.fqnm_invariants_get(h)
    b = F.fqnm_invariants_get_noalloc(h)
    assert a == b, (a, b)
    return b


def test_noalloc_matches_allocating_call_large_then_small():
    cases = [((1 << 26) + 12345, F.I32, F.BC_PERIODIC, 3, 1),   # 4096 blocks of > 16384 cells
             (100003, F.I64, F.BC_OUTFLOW, 17, 2),              # smaller: scratch reused
             (1, F.I32, F.BC_PERIODIC, 1, 3)]
    for n, itype, bc, steps, seed in cases:
        print("noalloc case", n, itype, bc, flush=True)
        h = _ctx_scalar(n, itype, bc, steps, seed)
        try:
            inv = _same(h)
            assert inv["steps_done"] == steps
            if bc == F.BC_PERIODIC:
                assert inv["ledger"] == [0]
        finally:
            F.fqnm_destroy(h)


def test_noalloc_euler_three_components_twice():
    for n in (40000, 2048):
        r = W.sod_request(n)
        prob = F.make_problem(F.FLUX_EULER_ROE_EF, r.delta, r.lam, n, itype=F.I64,
                              bc=F.BC_OUTFLOW, gamma=r.gamma)
        h = F.fqnm_create_from_field(prob, r.U0.ravel())
        try:
            F.fqnm_step(h, 50)
            inv = _same(h)
            assert inv["components"] == 3
        finally:
            F.fqnm_destroy(h)
