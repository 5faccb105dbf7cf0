"""GPU tests of the library's error behaviour and of the arithmetic it relies on:

* device FP64 division and square root, bit for bit against the host's
  correctly rounded ones, on 10^8 inputs (random bit patterns over every
  exponent range, special values) -- the Euler transfer is exact only if they are;
* an Euler state whose pressure turns non-positive (a strong rarefaction the
  Roe linearisation cannot follow) raises a sticky FQNM_ERR_RANGE at exactly
  the step where the oracle reports a non-finite state, and the steps before
  it are bit-exact;
* Lax-Friedrichs kinds, which have no exact integer maximum principle, refuse
  step counts whose reachable range could overflow the storage type
  (single grid, batch and server);
* the server counts the whole of a single-grid request's device memory,
  table included, against its budget;
* the block-tile kernels (plans 3, 4, 5) and the overlapping-window kernels
  (plans 7, 8) on table tiles spanning 2047 and 2048 levels, i.e. on both
  sides of their LDS-slice threshold, with both boundary kinds.
"""
import numpy as np
import pytest

import oracle as O
from paper_2604_06947_amd import fqnm as F
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    F.lib()


def test_fp64_div_sqrt_1e8_inputs():
    import torch
    rng = np.random.default_rng(2024)
    chunk, chunks = 4_000_000, 25
    st = torch.cuda.current_stream().cuda_stream
    specials = np.array([0.0, -0.0, 1.0, 2.0, 0.5, 3.0, 1e-300, 5e-324, 2.0 ** -1022,
                         1.7976931348623157e308, np.inf, -np.inf, 1e300, -1.0, 0.1, 1.4])
    checked = 0
    for c in range(chunks):
        bits = rng.integers(0, 2 ** 63, size=chunk, dtype=np.uint64)
        a = bits.view(np.float64).copy()                     # every exponent, positive
        b = rng.integers(0, 2 ** 64 - 1, size=chunk, dtype=np.uint64).view(np.float64).copy()
        if c == 0:
            a[:specials.size] = np.abs(specials)
            b[:specials.size] = specials[::-1]
        if c % 5 == 1:  # values of the size the Roe flux sees
            a = rng.uniform(1e-3, 10.0, chunk)
            b = rng.uniform(1e-7, 10.0, chunk) * rng.choice([-1.0, 1.0], chunk)
        da, db = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
        ds, dd = torch.empty_like(da), torch.empty_like(da)
        F.fqnm_fp64_selfcheck(da.data_ptr(), db.data_ptr(), ds.data_ptr(), dd.data_ptr(),
                              chunk, st)
        s, d = ds.cpu().numpy(), dd.cpu().numpy()
        with np.errstate(all="ignore"):
            rs, rd = np.sqrt(a), a / b
        for got, ref in ((s, rs), (d, rd)):
            nan = np.isnan(ref)
            assert np.array_equal(np.isnan(got), nan)
            assert np.array_equal(got[~nan].view(np.uint64), ref[~nan].view(np.uint64))
        checked += chunk
        del da, db, ds, dd
    assert checked >= 10 ** 8


def test_euler_nonpositive_pressure_is_a_sticky_range_error():
    left, right = (1.0, -2.0, 0.4), (1.0, 2.0, 0.4)  # two streams moving apart
    n = 512
    r = W.sod_request(n, left, right, kind=F.FLUX_EULER_ROE_EF)
    op = O.Problem(O.EULER_ROE_EF, r.delta, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
    q = np.stack([O.quantise(r.U0[c], r.delta) for c in range(3)])
    fail_at = None
    for s in range(1, 60):
        try:
            q = O.step_euler(op, q, 1)
        except O.OracleError:
            fail_at = s
            break
    assert fail_at is not None and fail_at >= 2
    good = O.step_euler(op, np.stack([O.quantise(r.U0[c], r.delta) for c in range(3)]),
                        fail_at - 1)
    prob = F.make_problem(F.FLUX_EULER_ROE_EF, r.delta, r.lam, n, bc=F.BC_OUTFLOW,
                          itype=F.I64, gamma=r.gamma)
    h = F.fqnm_create_from_field(prob, r.U0.ravel())
    try:
        F.fqnm_step(h, fail_at - 1)
        got = F.fqnm_get_state(h, prob).reshape(3, n)
        assert np.array_equal(got, good)
        F.fqnm_step(h, 1)
        with pytest.raises(F.FqnmError) as e:
            F.fqnm_get_state(h, prob)
        assert e.value.status == F.ERR_RANGE
        with pytest.raises(F.FqnmError) as e:
            F.fqnm_step(h, 1)
        assert e.value.status == F.ERR_RANGE
    finally:
        F.fqnm_destroy(h)
    # the same request through the server completes with that status
    srv = F.fqnm_server_create(64 << 20, 64)
    try:
        q0 = F.fqnm_quantise(r.U0.ravel(), r.delta, F.I64)
        out = np.empty_like(q0)
        F.fqnm_server_submit(srv, prob, q0, 40, out)
        F.fqnm_server_drain(srv, 60.0)
        comps = F.fqnm_server_poll(srv, 8)
    finally:
        F.fqnm_server_destroy(srv)
    assert len(comps) == 1 and comps[0]["status"] == F.ERR_RANGE


def lf_near_limit():
    """LF_LINEAR int32 (a = alpha = 1, dt/dx = 1) whose initial range sits 1000
    counts below what create accepts (5 |q| + 4 < 2^31 - 1 on the reachable
    range): with a drift of 2 counts per step, 500 steps remain."""
    n = 1000
    qa = (2 ** 31 - 5) // 5 - 1000
    q0 = W.random_states(n, -qa, qa, seed=17)
    q0[0], q0[1] = -qa, qa
    prob = F.make_problem(F.FLUX_LF_LINEAR, 1.0, 1.0, n, itype=F.I32, a=1.0, alpha=1.0,
                          eval_=F.EVAL_DIRECT)
    op = O.Problem(O.LF_LINEAR, 1.0, 1.0, width=32, a=1.0, alpha=1.0)
    return q0, prob, op


def test_lf_drift_is_refused_before_it_can_overflow():
    q0, prob, op = lf_near_limit()
    h = F.fqnm_create(prob, q0.astype(np.int32))
    try:
        F.fqnm_step(h, 400)
        with pytest.raises(F.FqnmError) as e:
            F.fqnm_step(h, 700)  # 1100 steps could reach past the checked range
        assert e.value.status == F.ERR_RANGE
        got = F.fqnm_get_state(h, prob).astype(np.int64)  # unchanged by the refused call
        assert np.array_equal(got, O.step(op, q0, 400))
        assert F.fqnm_invariants_get(h)["steps_done"] == 400
    finally:
        F.fqnm_destroy(h)
    with pytest.raises(F.FqnmError) as e:
        F.fqnm_batch_create([prob], [q0.astype(np.int32)], [1100])
    assert e.value.status == F.ERR_RANGE
    hb = F.fqnm_batch_create([prob], [q0.astype(np.int32)], [450])
    F.fqnm_batch_destroy(hb)
    srv = F.fqnm_server_create(64 << 20, 64)
    try:
        with pytest.raises(F.FqnmError) as e:
            F.fqnm_server_submit(srv, prob, q0.astype(np.int32), 1100,
                                 np.empty(q0.size, np.int32))
        assert e.value.status == F.ERR_RANGE
    finally:
        F.fqnm_server_destroy(srv)


def test_server_budget_counts_the_table_of_a_single_grid_request():
    budget = 64 << 20
    n, lam = 4096, 0.5
    delta = 1e-9
    prob = F.make_problem(F.FLUX_UPWIND, delta, lam, n, itype=F.I64, eval_=F.EVAL_LUT, a=1.0)
    op = O.Problem(O.UPWIND, delta, lam, width=64, a=1.0)
    big = W.random_states(n, -2_500_000, 2_500_000, seed=3)   # table of 5e6 x 16 B = 80 MB
    small = W.random_states(n, -1_000_000, 1_000_000, seed=4)  # table of 2e6 x 16 B = 32 MB
    srv = F.fqnm_server_create(budget, 64)
    try:
        with pytest.raises(F.FqnmError) as e:
            F.fqnm_server_submit(srv, prob, big, 100, np.empty(n, np.int64))
        assert e.value.status == F.ERR_OOM
        out = np.empty(n, np.int64)
        F.fqnm_server_submit(srv, prob, small, 300, out)
        F.fqnm_server_drain(srv, 60.0)
        comps = F.fqnm_server_poll(srv, 8)
        stats = F.fqnm_server_stats_get(srv)
    finally:
        F.fqnm_server_destroy(srv)
    assert len(comps) == 1 and comps[0]["status"] == 0
    assert np.array_equal(out, O.step(op, small, 300))
    assert 32_000_000 < stats["peak_bytes"] <= budget


def spans_pattern(n, lo, hi_a, hi_b, seed):
    """Every 16th cell holds lo; every 16th (offset 8) holds hi_a in the first
    half and hi_b in the second; the rest is random in [lo, hi_a]."""
    rng = np.random.default_rng(seed)
    half = n // 2
    q0 = rng.integers(lo, hi_a + 1, n)
    q0[0::16] = lo
    q0[8:half:16] = hi_a
    q0[half + 8 - half % 16::16] = hi_b
    return q0


@pytest.mark.parametrize("bc", [F.BC_PERIODIC, F.BC_OUTFLOW])
def test_block_tiles_at_their_slice_threshold(bc):
    """Workgroup tiles stage the table slice in LDS when their states span
    fewer than 2048 levels and evaluate the maps directly otherwise; every
    tile here spans 2047 (first half) or 2048 levels (second half)."""
    n = 24_007
    q0 = spans_pattern(n, -1024, 1023, 1024, seed=91)
    delta = 1e-3
    prob = F.make_problem(F.FLUX_BURGERS_EO, delta, 0.45 / (1024 * delta), n, bc=bc,
                          itype=F.I32, eval_=F.EVAL_LUT)
    op = O.Problem(O.BURGERS_EO, delta, 0.45 / (1024 * delta), bc=bc, width=32)
    ref, led = O.step(op, q0, 120, return_ledger=True)
    plans = [(F.KERNEL_TBLOCK_B2, 4, 24), (F.KERNEL_TBLOCK_B4, 4, 48),
             (F.KERNEL_TBLOCK_B8, 4, 64), (F.KERNEL_TBLOCK_B4, 8, 96)]
    if bc == F.BC_PERIODIC:
        plans += [(F.KERNEL_TBLOCK_WG4, 4, 48), (F.KERNEL_TBLOCK_WG8, 2, 64)]
    for plan in plans:
        h = F.fqnm_create(prob, q0.astype(np.int32))
        try:
            F.fqnm_set_plan(h, *plan)
            F.fqnm_step(h, 120)
            got = F.fqnm_get_state(h, prob).astype(np.int64)
            inv = F.fqnm_invariants_get(h)
        finally:
            F.fqnm_destroy(h)
        assert np.array_equal(got, ref), plan
        assert inv["ledger"][0] == led
