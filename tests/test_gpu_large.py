"""Grids of more than 2^31 cells: every cell index, tile index and byte offset
of the stepping, reduction and copy kernels must be 64-bit.

The state is filled on the device with seeded values and handed to the
library in place (fqnm_create_on_device, so no 8-16 GiB host transfer).  After
the steps, cells sampled across the grid (both ends, both sides of index
2^31, seeded others) are compared with the oracle run on the window of
initial states each of them depends on: on a periodic grid a cell after s
steps depends only on the 2s+1 cells around it (three-cell stencil), so the
middle cell of a window of radius r >= s comes out exact whatever the
window's own boundary does.  The exact sum is checked against the initial
sum (conservation, eq:exact_conservation), modulo 2^64 as torch sums.

Int32 states are random walks (steps of -1, 0, +1), smooth enough for the
tables' LDS slices; int64 states are uniform over a range past 2^32."""
import numpy as np
import pytest

import oracle as O
from paper_2604_06947_amd import fqnm as F

pytestmark = pytest.mark.gpu

N = 2 ** 31 + 333
DELTA = 1e-3

# name: flux, state type, table mode, plan (None: the library's default), steps
CASES = {
    "upwind_i32": (F.FLUX_UPWIND, F.I32, False, None, 60),
    "upwind_i32_stream": (F.FLUX_UPWIND, F.I32, False, (F.KERNEL_STREAM, 4, 1), 5),
    "eo_table_i32": (F.FLUX_BURGERS_EO, F.I32, True, None, 60),
    "upwind_i64": (F.FLUX_UPWIND, F.I64, False, None, 60),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    F.lib()


def initial_state(itype, seed):
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    if itype == F.I32:
        steps = torch.randint(-1, 2, (N,), generator=g, device="cuda", dtype=torch.int8)
        t = torch.cumsum(steps, 0, dtype=torch.int64)
        del steps
        t = t.to(torch.int32)
    else:
        t = torch.randint(-(2 ** 33), 2 ** 33, (N,), generator=g, device="cuda",
                          dtype=torch.int64)
    torch.cuda.synchronize()
    return t


@pytest.mark.parametrize("case", list(CASES))
def test_grid_beyond_2_to_31_cells(case):
    import torch
    flux, itype, lut, plan, steps = CASES[case]
    print("large grid", case, N, steps, flush=True)
    t = initial_state(itype, seed=2031)
    qmax = int(t.abs().max())
    if flux == F.FLUX_UPWIND:
        a = 1.0 if itype == F.I32 else -0.7
        lam, kind = 0.9 / abs(a), O.UPWIND
    else:
        a, lam, kind = 1.0, 0.45 / (DELTA * qmax), O.BURGERS_EO
    prob = F.make_problem(flux, DELTA, lam, N, itype=itype,
                          eval_=F.EVAL_LUT if lut else F.EVAL_DIRECT, a=a)
    op = O.Problem(kind, DELTA, lam, width=32 if itype == F.I32 else 64, a=a)

    rng = np.random.default_rng(31)
    centres = np.unique(np.concatenate([[0, 1, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + 1, N - 1],
                                        rng.integers(0, N, 26)]))
    r = steps + 2
    idx = (centres[:, None] + np.arange(-r, r + 1)[None, :]) % N
    win = t[torch.from_numpy(idx.reshape(-1)).to("cuda")].cpu().numpy()
    win = win.astype(np.int64).reshape(idx.shape)
    total = int(t.sum(dtype=torch.int64))

    stream = torch.cuda.current_stream().cuda_stream
    h = F.fqnm_create_on_device(prob, t.data_ptr(), stream)
    try:
        if plan is not None:
            F.fqnm_set_plan(h, *plan)
        F.fqnm_step(h, steps)
        inv = F.fqnm_invariants_get(h)
        torch.cuda.synchronize()
        got = t[torch.from_numpy(centres).to("cuda")].cpu().numpy().astype(np.int64)
    finally:
        F.fqnm_destroy(h)
    del t
    torch.cuda.empty_cache()

    assert inv["steps_done"] == steps
    assert inv["sum"][0] % 2 ** 64 == total % 2 ** 64
    for k, c in enumerate(centres):
        ref = O.step(op, win[k], steps)[r]
        assert got[k] == ref, (case, int(c))
