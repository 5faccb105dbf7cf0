"""GPU parity of the single-grid stepper against the CPU oracle, through the C ABI.

Integer states must match bit for bit (the method is deterministic integer
arithmetic with fixed-order FP64 maps, so there is exactly one correct
trajectory).  Sizes span several tiles and a ragged tail; every launch plan
must give the same bytes, which also catches halo and race mistakes.
"""
import numpy as np
import pytest

import oracle as O
from paper_2604_06947_amd import fqnm as F
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.gpu

KIND_F2O = {F.FLUX_UPWIND: O.UPWIND, F.FLUX_BURGERS_EO: O.BURGERS_EO,
            F.FLUX_BURGERS_GODUNOV: O.BURGERS_GODUNOV, F.FLUX_LF_LINEAR: O.LF_LINEAR,
            F.FLUX_LF_BURGERS: O.LF_BURGERS, F.FLUX_BURGERS_MURMAN_ROE: O.BURGERS_MURMAN_ROE,
            F.FLUX_EULER_ROE: O.EULER_ROE, F.FLUX_EULER_ROE_EF: O.EULER_ROE_EF}

PLANS32 = [(F.KERNEL_STREAM, 4, 1), (F.KERNEL_STREAM, 8, 1), (F.KERNEL_STREAM, 16, 1),
           (F.KERNEL_TBLOCK, 4, 1), (F.KERNEL_TBLOCK, 4, 4), (F.KERNEL_TBLOCK, 8, 8),
           (F.KERNEL_TBLOCK, 16, 32), (F.KERNEL_TBLOCK, 16, 96), (F.KERNEL_TBLOCK, 8, 64),
           (F.KERNEL_TBLOCK_IL, 4, 16), (F.KERNEL_TBLOCK_IL, 8, 64), (F.KERNEL_TBLOCK_IL, 16, 100),
           (F.KERNEL_TBLOCK_B2, 4, 8), (F.KERNEL_TBLOCK_B4, 4, 48), (F.KERNEL_TBLOCK_B8, 8, 64)]
PLANS64 = [(F.KERNEL_STREAM, 2, 1), (F.KERNEL_STREAM, 8, 1), (F.KERNEL_TBLOCK, 2, 2),
           (F.KERNEL_TBLOCK, 4, 8), (F.KERNEL_TBLOCK, 8, 16), (F.KERNEL_TBLOCK, 8, 48),
           (F.KERNEL_TBLOCK_IL, 4, 8), (F.KERNEL_TBLOCK_IL, 8, 64),
           (F.KERNEL_TBLOCK_B2, 2, 6), (F.KERNEL_TBLOCK_B4, 8, 24), (F.KERNEL_TBLOCK_B8, 4, 40)]
# 64-bit upwind maps evaluated directly also run 16 cells per lane (kernel 1)
PLANS64_UPWIND = [(F.KERNEL_TBLOCK, 16, 1), (F.KERNEL_TBLOCK, 16, 40), (F.KERNEL_TBLOCK, 16, 100)]
TWO_POINT = (F.FLUX_BURGERS_GODUNOV, F.FLUX_BURGERS_MURMAN_ROE)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    F.lib()


def gpu_run(prob, q0=None, u0=None, steps=0, plan=None):
    h = F.fqnm_create(prob, q0) if u0 is None else F.fqnm_create_from_field(prob, u0)
    try:
        if plan is not None:
            F.fqnm_set_plan(h, *plan)
        F.fqnm_step(h, steps)
        q = F.fqnm_get_state(h, prob).astype(np.int64)
        inv = F.fqnm_invariants_get(h)
    finally:
        F.fqnm_destroy(h)
    return q, inv


def oracle_problem(prob):
    return O.Problem(KIND_F2O[prob.flux], prob.delta, prob.lambda_, bc=prob.bc,
                     width=32 if prob.itype == F.I32 else 64, a=prob.a, alpha=prob.alpha,
                     gamma=prob.gamma)


def plans_for(itype, flux=None):
    plans = PLANS32 if itype == F.I32 else PLANS64
    if flux in TWO_POINT:  # interleaved tiles serve split kinds only
        plans = [p for p in plans if p[0] != F.KERNEL_TBLOCK_IL]
    return plans


# ---------------------------------------------------------------------------
def test_w1_advection_square_every_plan():
    w = W.w1_advection_square()
    ref = O.step(O.Problem(O.UPWIND, w.delta, w.lam, width=32, a=1.0),
                 O.quantise(w.u0, w.delta, 32), w.steps)
    prob = F.make_problem(F.FLUX_UPWIND, w.delta, w.lam, w.n, itype=F.I32, a=1.0)
    for plan in PLANS32:
        q, inv = gpu_run(prob, u0=w.u0, steps=w.steps, plan=plan)
        assert np.array_equal(q, ref), plan
        assert inv["sum"][0] == int(ref.sum())


def make_case(flux, bc, itype, n, seed, a=1.0, alpha=0.0, lut=False):
    u0 = W.random_smooth_step(n, seed=seed, b=0.1)
    delta = 1e-4 if itype == F.I32 else 1e-7
    umax = float(np.max(np.abs(u0)))
    if flux == F.FLUX_UPWIND:
        lam = 0.77 / abs(a)
    elif flux in (F.FLUX_LF_LINEAR, F.FLUX_LF_BURGERS):
        alpha = max(abs(a), umax) * 1.25 if flux == F.FLUX_LF_LINEAR else umax * 1.25
        lam = 0.8 / alpha
    else:
        lam = 0.45 / umax
    return u0, F.make_problem(flux, delta, lam, n, bc=bc, itype=itype,
                              eval_=F.EVAL_LUT if lut else F.EVAL_DIRECT, a=a, alpha=alpha)


KINDS = [(F.FLUX_UPWIND, 1.0, False), (F.FLUX_UPWIND, -0.9, False), (F.FLUX_UPWIND, 1.0, True),
         (F.FLUX_UPWIND, -0.9, True),
         (F.FLUX_BURGERS_EO, 1.0, False), (F.FLUX_BURGERS_EO, 1.0, True),
         (F.FLUX_BURGERS_GODUNOV, 1.0, False), (F.FLUX_BURGERS_MURMAN_ROE, 1.0, False),
         (F.FLUX_LF_LINEAR, 0.6, False), (F.FLUX_LF_BURGERS, 1.0, False)]


@pytest.mark.parametrize("flux,a,lut", KINDS)
@pytest.mark.parametrize("bc", [F.BC_PERIODIC, F.BC_OUTFLOW])
@pytest.mark.parametrize("itype", [F.I32, F.I64])
def test_kind_parity_all_plans(flux, a, lut, bc, itype):
    n, steps = 5003, 150
    u0, prob = make_case(flux, bc, itype, n, seed=100 + flux, a=a, lut=lut)
    op = oracle_problem(prob)
    q0 = O.quantise(u0, prob.delta, op.width)
    ref, led = O.step(op, q0, steps, return_ledger=True)
    plans = plans_for(itype, flux)
    if itype == F.I64 and flux == F.FLUX_UPWIND and not lut:
        plans = plans + PLANS64_UPWIND
    for plan in plans:
        q, inv = gpu_run(prob, u0=u0, steps=steps, plan=plan)
        assert np.array_equal(q, ref), plan
        assert inv["ledger"][0] == led
        assert inv["sum"][0] == int(ref.sum())


@pytest.mark.parametrize("flux,a", [(F.FLUX_BURGERS_EO, 1.0), (F.FLUX_UPWIND, 1.0),
                                    (F.FLUX_UPWIND, -0.9)])
@pytest.mark.parametrize("bc", [F.BC_PERIODIC, F.BC_OUTFLOW])
def test_table_clamped_and_certified_reads_agree(flux, a, bc, monkeypatch):
    """Int32 tables certify the maximum principle at build, and kernel 1 then
    reads its LDS slices without clamping; with FQNM_TABLE_CLAMPED set it
    takes the clamped reads instead.  Both give the oracle's integers."""
    n, steps = 20011, 130
    u0, prob = make_case(flux, bc, F.I32, n, seed=211, a=a, lut=True)
    op = oracle_problem(prob)
    ref, led = O.step(op, O.quantise(u0, prob.delta, 32), steps, return_ledger=True)
    for clamped in (False, True):
        if clamped:
            monkeypatch.setenv("FQNM_TABLE_CLAMPED", "1")
        else:
            monkeypatch.delenv("FQNM_TABLE_CLAMPED", raising=False)
        for plan in ((F.KERNEL_TBLOCK, 4, 40), (F.KERNEL_TBLOCK, 4, 52), (F.KERNEL_TBLOCK, 8, 64),
                     (F.KERNEL_TBLOCK, 16, 96)):
            q, inv = gpu_run(prob, u0=u0, steps=steps, plan=plan)
            assert np.array_equal(q, ref), (clamped, plan)
            assert inv["ledger"][0] == led


@pytest.mark.parametrize("bc", [F.BC_PERIODIC, F.BC_OUTFLOW])
@pytest.mark.parametrize("lo", [-192, -256])
def test_table_tiles_at_the_slice_threshold(bc, lo):
    """Int32 tables: a wavefront copies its tile's slice of the table into LDS
    when the tile's states span fewer than 512 levels and otherwise evaluates
    the split maps the table was built from.  Every 16th cell holds lo and
    every 16th (offset 8) holds -lo - 1 in the first half of the grid and -lo
    in the second, so every tile spans exactly 2|lo| - 1 or 2|lo| levels:
    with lo = -256 both sides of the threshold, with lo = -192 slices well
    inside it.  Both must give the oracle's integers, for the single-launch
    and the persistent plans."""
    rng = np.random.default_rng(77)
    n = 176 * 12
    half = n // 2
    hi = -lo
    q0 = np.concatenate([rng.integers(lo, hi, half), rng.integers(lo, hi + 1, n - half)])
    q0[0::16] = lo
    q0[8:half:16] = hi - 1
    q0[half + 8 - half % 16::16] = hi
    delta = 1e-3
    prob = F.make_problem(F.FLUX_BURGERS_EO, delta, 0.45 / (hi * delta), n, bc=bc,
                          itype=F.I32, eval_=F.EVAL_LUT)
    op = oracle_problem(prob)
    ref, led = O.step(op, q0, 100, return_ledger=True)
    plans = [None, (F.KERNEL_TBLOCK, 4, 40), (F.KERNEL_TBLOCK, 4, 52), (F.KERNEL_TBLOCK, 4, 8),
             (F.KERNEL_TBLOCK, 8, 16), (F.KERNEL_TBLOCK, 16, 32)]
    if bc == F.BC_PERIODIC:
        plans += [(10, 4, 40), (10, 4, 8), (10, 8, 24)]
    for plan in plans:
        q, inv = gpu_run(prob, q0=q0.astype(np.int32), steps=100, plan=plan)
        assert np.array_equal(q, ref), plan
        assert inv["ledger"][0] == led


@pytest.mark.parametrize("n", [1, 2, 3, 7, 63, 64, 65, 127, 959, 960, 961, 1985])
@pytest.mark.parametrize("bc", [F.BC_PERIODIC, F.BC_OUTFLOW])
def test_edge_sizes(n, bc):
    for flux in (F.FLUX_UPWIND, F.FLUX_BURGERS_EO, F.FLUX_BURGERS_GODUNOV):
        u0, prob = make_case(flux, bc, F.I32, n, seed=7 + n, lut=False)
        op = oracle_problem(prob)
        q0 = O.quantise(u0, prob.delta, 32)
        for steps in (0, 1, 37):
            ref = O.step(op, q0, steps)
            plans = [(F.KERNEL_STREAM, 4, 1), (F.KERNEL_TBLOCK, 4, 4), (F.KERNEL_TBLOCK, 16, 32),
                     (F.KERNEL_TBLOCK_B4, 4, 12), (F.KERNEL_TBLOCK_B8, 8, 64)]
            if flux not in TWO_POINT:
                plans.append((F.KERNEL_TBLOCK_IL, 4, 16))
            for plan in plans:
                q, _ = gpu_run(prob, q0=q0.astype(np.int32), steps=steps, plan=plan)
                assert np.array_equal(q, ref), (flux, steps, plan)


def test_quantise_and_reconstruct_match_oracle():
    rng = np.random.default_rng(5)
    n = 10007
    u0 = rng.uniform(-3, 3, n)
    u0[:8] = np.array([2.5, 3.5, -2.5, -0.5, 0.5, 1.5, 7.25, -7.75]) * 2.0 ** -10  # ties
    for itype, width in ((F.I32, 32), (F.I64, 64)):
        delta = 2.0 ** -10
        prob = F.make_problem(F.FLUX_UPWIND, delta, 0.5, n, itype=itype)
        h = F.fqnm_create_from_field(prob, u0)
        try:
            q = F.fqnm_get_state(h, prob).astype(np.int64)
            u = F.fqnm_reconstruct(h, prob)
        finally:
            F.fqnm_destroy(h)
        assert np.array_equal(q, O.quantise(u0, delta, width))
        assert np.array_equal(u, O.reconstruct(q, delta))


def test_invariants_match_oracle():
    u0, prob = make_case(F.FLUX_BURGERS_EO, F.BC_PERIODIC, F.I64, 70001, seed=9)
    q0 = O.quantise(u0, prob.delta, 64)
    h = F.fqnm_create(prob, q0)
    try:
        F.fqnm_step(h, 100)
        inv = F.fqnm_invariants_get(h)
        q = F.fqnm_get_state(h, prob)
    finally:
        F.fqnm_destroy(h)
    ref = O.invariants(q, periodic=True)
    assert inv["sum"][0] == ref["sum"] == int(q0.sum())
    assert inv["min"][0] == ref["min"] and inv["max"][0] == ref["max"]
    assert inv["tv"][0] == ref["tv"]
    assert inv["steps_done"] == 100


def test_checkpoint_resume_bitexact():
    u0, prob = make_case(F.FLUX_BURGERS_EO, F.BC_OUTFLOW, F.I32, 20000, seed=3, lut=True)
    qa, _ = gpu_run(prob, u0=u0, steps=333)
    q1, _ = gpu_run(prob, u0=u0, steps=120)
    qb, _ = gpu_run(prob, q0=q1.astype(np.int32), steps=213)
    assert np.array_equal(qa, qb)


def test_create_on_device_keeps_state_in_tensor():
    import torch
    u0, prob = make_case(F.FLUX_UPWIND, F.BC_PERIODIC, F.I32, 4099, seed=11)
    q0 = O.quantise(u0, prob.delta, 32)
    t = torch.tensor(q0.astype(np.int32), device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    h = F.fqnm_create_on_device(prob, t.data_ptr(), stream)
    try:
        F.fqnm_set_plan(h, F.KERNEL_TBLOCK, 8, 7)
        F.fqnm_step(h, 45)  # an odd number of launches
        torch.cuda.synchronize()
        got = t.cpu().numpy().astype(np.int64)
    finally:
        F.fqnm_destroy(h)
    assert np.array_equal(got, O.step(oracle_problem(prob), q0, 45))


@pytest.mark.parametrize("flux,itype,lut,n,vec,depth", [
    (F.FLUX_UPWIND, F.I32, False, 1024, 4, 120), (F.FLUX_BURGERS_EO, F.I32, True, 1024, 4, 120),
    (F.FLUX_UPWIND, F.I32, False, 8192, 4, 120), (F.FLUX_UPWIND, F.I32, False, 65536, 4, 96),
    (F.FLUX_UPWIND, F.I32, False, 262144, 4, 52), (F.FLUX_UPWIND, F.I32, False, 1 << 20, 4, 24),
    (F.FLUX_UPWIND, F.I64, False, 1024, 4, 120), (F.FLUX_UPWIND, F.I64, False, 262144, 4, 52),
    (F.FLUX_UPWIND, F.I64, False, 1 << 20, 16, 200),
    (F.FLUX_BURGERS_EO, F.I64, False, 65536, 4, 96)])
def test_small_grids_take_deep_passes(flux, itype, lut, n, vec, depth):
    """The default plan of a single grid (no tuned plan cached): the first of
    4-cell lanes at 120..52 steps per pass (then, for 64-bit upwind states,
    16-cell lanes at 200) whose tiles number at most 1.75 per SIMD (1024 SIMDs
    on MI355X) and whose pass is deeper than the default; bit-exact against
    the oracle."""
    u0, prob = make_case(flux, F.BC_PERIODIC, itype, n, seed=29, lut=lut)
    width = 32 if itype == F.I32 else 64
    h = F.fqnm_create_from_field(prob, u0)
    try:
        pl = F.fqnm_get_plan(h)
        F.fqnm_step(h, 250)
        q = F.fqnm_get_state(h, prob).astype(np.int64)
    finally:
        F.fqnm_destroy(h)
    assert (pl["kernel"], pl["vec"], pl["depth"]) == (F.KERNEL_TBLOCK, vec, depth)
    ref = O.step(oracle_problem(prob), O.quantise(u0, prob.delta, width), 250)
    assert np.array_equal(q, ref)


@pytest.mark.parametrize("n", [777, 2112])
def test_passes_deeper_than_tiles_on_outflow_grids(n):
    """Passes deeper than a tile is wide: the windows of several tiles reach
    past each end of an outflow grid, and only the tiles holding cell 0 and
    cell n-1 may count the transfers across the ends.  States and ledger
    against the oracle for every lane-contiguous, workgroup and interleaved
    kernel with tiles narrower than their halo."""
    plans = [(F.KERNEL_TBLOCK, 4, 120), (F.KERNEL_TBLOCK, 8, 240),
             (F.KERNEL_TBLOCK_B4, 4, 400), (F.KERNEL_TBLOCK_IL, 8, 192)]
    for flux, a, lut in [(F.FLUX_UPWIND, 1.0, False), (F.FLUX_UPWIND, -0.9, True),
                         (F.FLUX_BURGERS_EO, 1.0, True), (F.FLUX_BURGERS_EO, 1.0, False),
                         (F.FLUX_BURGERS_GODUNOV, 1.0, False)]:
        u0, prob = make_case(flux, F.BC_OUTFLOW, F.I32, n, seed=41, a=a, lut=lut)
        op = oracle_problem(prob)
        q0 = O.quantise(u0, prob.delta, 32)
        ref, led = O.step(op, q0, 300, return_ledger=True)
        for plan in plans:
            if plan[0] == F.KERNEL_TBLOCK_IL and flux in TWO_POINT:
                continue
            q, inv = gpu_run(prob, q0=q0.astype(np.int32), steps=300, plan=plan)
            assert np.array_equal(q, ref), (flux, lut, plan)
            assert inv["ledger"][0] == led, (flux, lut, plan)


def test_autotune_small_grid_considers_deep_passes():
    """On a grid of one or two tiles per SIMD the autotuner also times passes
    deeper than a tile is wide (up to 120 steps in 4-cell lanes): the plan it
    keeps is a blocked one at least 52 steps deep, and steps the grid (outflow
    ends, so the ledger too) bit-exactly."""
    w = W.w1_advection_square()
    prob = F.make_problem(F.FLUX_UPWIND, w.delta, w.lam, w.n, itype=F.I32, a=w.a,
                          bc=F.BC_OUTFLOW)
    h = F.fqnm_create_from_field(prob, w.u0)
    try:
        F.fqnm_autotune(h, 240)
        plan = F.fqnm_get_plan(h)
        F.fqnm_step(h, w.steps)
        q = F.fqnm_get_state(h, prob).astype(np.int64)
        inv = F.fqnm_invariants_get(h)
    finally:
        F.fqnm_destroy(h)
    assert plan["kernel"] != F.KERNEL_STREAM and plan["depth"] >= 52, plan
    ref, led = O.step(oracle_problem(prob), O.quantise(w.u0, w.delta, 32), w.steps,
                      return_ledger=True)
    assert np.array_equal(q, ref) and inv["ledger"][0] == led


def test_autotune_then_parity():
    w = W.w2_burgers_step(n=1 << 16, steps=300)
    prob = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam, w.n, itype=F.I32,
                          eval_=F.EVAL_LUT)
    h = F.fqnm_create_from_field(prob, w.u0)
    try:
        F.fqnm_autotune(h, 64)
        plan = F.fqnm_get_plan(h)
        F.fqnm_step(h, w.steps)
        q = F.fqnm_get_state(h, prob).astype(np.int64)
        inv = F.fqnm_invariants_get(h)
    finally:
        F.fqnm_destroy(h)
    assert plan["eval"] == F.EVAL_LUT and inv["steps_done"] == w.steps
    ref = O.step(O.Problem(O.BURGERS_EO, w.delta, w.lam, width=32),
                 O.quantise(w.u0, w.delta, 32), w.steps)
    assert np.array_equal(q, ref)


def test_interleaved_plan_rejected_for_two_point_kinds():
    u0, prob = make_case(F.FLUX_BURGERS_GODUNOV, F.BC_PERIODIC, F.I32, 1000, seed=1)
    h = F.fqnm_create_from_field(prob, u0)
    try:
        with pytest.raises(F.FqnmError) as e:
            F.fqnm_set_plan(h, F.KERNEL_TBLOCK_IL, 8, 16)
        assert e.value.status == F.ERR_ARG
    finally:
        F.fqnm_destroy(h)


@pytest.mark.parametrize("bad", ["cfl", "lut_godunov", "range", "lut_range", "abi", "euler_i32",
                                 "n0"])
def test_create_rejects_invalid_problems(bad):
    n = 100
    q0 = np.zeros(n, np.int32)
    prob = F.make_problem(F.FLUX_UPWIND, 1e-3, 0.5, n, itype=F.I32)
    want = F.ERR_ARG
    if bad == "cfl":
        prob.lambda_ = 1.5
        want = F.ERR_CFL
    elif bad == "lut_godunov":
        prob.flux = F.FLUX_BURGERS_GODUNOV
        prob.eval = F.EVAL_LUT
    elif bad == "range":
        q0 = np.full(n, 2 ** 31 - 10, np.int32)
        want = F.ERR_RANGE
    elif bad == "lut_range":  # a table over 2^28 or more states is refused before allocation
        prob.eval = F.EVAL_LUT
        q0[0], q0[1] = -(2 ** 27), 2 ** 27
        want = F.ERR_RANGE
    elif bad == "abi":
        prob.abi_version = 99
    elif bad == "euler_i32":
        prob.flux = F.FLUX_EULER_ROE
        q0 = np.zeros(3 * n, np.int32)
    elif bad == "n0":
        prob.n = 0
        q0 = np.zeros(0, np.int32)
    with pytest.raises((F.FqnmError, ValueError)) as e:
        F.fqnm_create(prob, q0)
    if isinstance(e.value, F.FqnmError):
        assert e.value.status == want


# ---------------------------------------------------------------------------
# Full-size workloads: sampled cells against the oracle.  A cell after s
# steps depends only on the 2s+1 cells around it, so the oracle steps that
# window (any boundary) and its centre is exact.
# ---------------------------------------------------------------------------
def window_centre(op, q0, i, s):
    n = q0.size
    idx = np.arange(i - s, i + s + 1) % n
    win = O.Problem(op.kind, op.delta, op.lam, bc=O.OUTFLOW, width=op.width, a=op.a,
                    alpha=op.alpha)
    return int(O.step(win, q0[idx], s)[s])


def test_w2_burgers_full_size_sampled():
    from paper_2604_06947_amd import plans
    w = W.w2_burgers_step()
    prob = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam, w.n, itype=F.I32,
                          eval_=F.EVAL_LUT)
    q, inv = gpu_run(prob, u0=w.u0, steps=w.steps, plan=plans.BENCH_PLAN_W2)
    q0 = O.quantise(w.u0, w.delta, 32)
    op = O.Problem(O.BURGERS_EO, w.delta, w.lam, width=32)
    assert inv["sum"][0] == int(q0.sum())
    assert q0.min() <= q.min() and q.max() <= q0.max()
    rng = np.random.default_rng(2024)
    xs = int(np.argmax(np.diff(q0) > 10000))  # near the seeded step
    for i in [0, w.n - 1, xs, xs + 1] + list(rng.integers(0, w.n, 2)):
        assert q[i] == window_centre(op, q0, int(i), w.steps), i


# Workgroup tiles with overlapping wavefront windows (int32 tables, periodic):
# depths below, at and above the refresh period, the largest allowed depth,
# a step count that ends on a partial pass; grids smaller than one window,
# one workgroup, several workgroups with a ragged tail; and states whose tile
# range is too wide for the shared table slice (the global-table path).
WG_PLANS = [(F.KERNEL_TBLOCK_WG4, 2, 5), (F.KERNEL_TBLOCK_WG4, 2, 8), (F.KERNEL_TBLOCK_WG4, 4, 48),
            (F.KERNEL_TBLOCK_WG8, 2, 24), (F.KERNEL_TBLOCK_WG8, 4, 96), (F.KERNEL_TBLOCK_WG4, 2, 112),
            (F.KERNEL_TBLOCK_WG8, 4, 17), (F.KERNEL_TBLOCK_WG4, 4, 240)]


@pytest.mark.parametrize("flux,a", [(F.FLUX_UPWIND, 1.0), (F.FLUX_UPWIND, -0.9),
                                    (F.FLUX_BURGERS_EO, 1.0)])
@pytest.mark.parametrize("n,amp", [(1, 1.0), (7, 1.0), (130, 1.0), (1000, 1.0), (5003, 1.0),
                                   (40000, 0.02), (40000, 1.0)])
def test_overlapping_window_tiles(flux, a, n, amp):
    u0, prob = make_case(flux, F.BC_PERIODIC, F.I32, n, seed=300 + n, a=a, lut=True)
    u0 = u0 * amp
    op = oracle_problem(prob)
    q0 = O.quantise(u0, prob.delta, 32)
    steps = 251
    ref = O.step(op, q0, steps)
    for plan in WG_PLANS:
        q, inv = gpu_run(prob, q0=q0.astype(np.int32), steps=steps, plan=plan)
        assert np.array_equal(q, ref), plan
        assert inv["sum"][0] == int(q0.sum())


def test_overlapping_window_tiles_refused_elsewhere():
    for bc, lut, itype in [(F.BC_OUTFLOW, True, F.I32), (F.BC_PERIODIC, False, F.I32),
                           (F.BC_PERIODIC, True, F.I64)]:
        u0, prob = make_case(F.FLUX_BURGERS_EO, bc, itype, 300, seed=1, lut=lut)
        h = F.fqnm_create_from_field(prob, u0)
        try:
            with pytest.raises(F.FqnmError):
                F.fqnm_set_plan(h, F.KERNEL_TBLOCK_WG4, 4, 48)
        finally:
            F.fqnm_destroy(h)
    u0, prob = make_case(F.FLUX_BURGERS_EO, F.BC_PERIODIC, F.I32, 300, seed=1, lut=True)
    h = F.fqnm_create_from_field(prob, u0)
    try:
        for bad in [(F.KERNEL_TBLOCK_WG4, 8, 48), (F.KERNEL_TBLOCK_WG8, 2, 113)]:
            with pytest.raises(F.FqnmError):
                F.fqnm_set_plan(h, *bad)
    finally:
        F.fqnm_destroy(h)


def test_w2_full_size_overlapping_windows_sampled():
    w = W.w2_burgers_step()
    prob = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam, w.n, itype=F.I32,
                          eval_=F.EVAL_LUT)
    q0 = O.quantise(w.u0, w.delta, 32)
    op = O.Problem(O.BURGERS_EO, w.delta, w.lam, width=32)
    xs = int(np.argmax(np.diff(q0) > 10000))  # near the seeded step
    rng = np.random.default_rng(2025)
    pts = [0, w.n - 1, xs, xs + 1] + list(rng.integers(0, w.n, 2))
    refs = {i: window_centre(op, q0, int(i), w.steps) for i in pts}
    for plan in [(F.KERNEL_TBLOCK_WG8, 4, 96), (F.KERNEL_TBLOCK_WG4, 2, 64)]:
        q, inv = gpu_run(prob, u0=w.u0, steps=w.steps, plan=plan)
        assert inv["sum"][0] == int(q0.sum())
        for i in pts:
            assert q[i] == refs[i], (plan, i)


@pytest.mark.parametrize("r", [1e-2, 1e-3, 1e-4])
@pytest.mark.parametrize("which", ["blocked", "streaming"])
def test_w3_nyquist_full_size_sampled(r, which):
    # both plans the benchmark times on this workload
    from paper_2604_06947_amd import plans
    plan = plans.BENCH_PLAN_W3 if which == "blocked" else plans.STREAM_PLAN_W3
    w = W.w3_nyquist_advection(r=r)
    prob = F.make_problem(F.FLUX_UPWIND, w.delta, w.lam, w.n, itype=F.I64, a=1.0)
    q, inv = gpu_run(prob, u0=w.u0, steps=w.steps, plan=plan)
    q0 = O.quantise(w.u0, w.delta, 64)
    assert inv["sum"][0] == int(q0.sum())
    op = O.Problem(O.UPWIND, w.delta, w.lam, width=64, a=1.0)
    rng = np.random.default_rng(int(1 / r))
    for i in [0, 1, w.n - 1] + list(rng.integers(0, w.n, 5)):
        assert q[i] == window_centre(op, q0, int(i), w.steps), i


def test_w3_reduced_bitexact():
    w = W.w3_nyquist_advection(r=1e-3, n=1 << 16, steps=300)
    prob = F.make_problem(F.FLUX_UPWIND, w.delta, w.lam, w.n, itype=F.I64, a=1.0)
    ref = O.step(O.Problem(O.UPWIND, w.delta, w.lam, width=64, a=1.0),
                 O.quantise(w.u0, w.delta, 64), w.steps)
    for plan in PLANS64 + PLANS64_UPWIND:
        q, _ = gpu_run(prob, u0=w.u0, steps=w.steps, plan=plan)
        assert np.array_equal(q, ref), plan


@pytest.mark.parametrize("n", [1, 2, 7, 63, 1023, 1024, 1025, 2047, 4099])
@pytest.mark.parametrize("bc", [F.BC_PERIODIC, F.BC_OUTFLOW])
@pytest.mark.parametrize("a", [1.0, -0.9])
def test_int64_upwind_wide_tiles_edge_sizes(n, bc, a):
    """16 cells per lane (1024-cell windows, stepped as exact doubles on plain
    windows, as integers on windows at outflow ends) on grids smaller than,
    equal to and just above one window."""
    u0, prob = make_case(F.FLUX_UPWIND, bc, F.I64, n, seed=300 + n, a=a)
    op = oracle_problem(prob)
    q0 = O.quantise(u0, prob.delta, 64)
    for steps in (0, 1, 37):
        ref, led = O.step(op, q0, steps, return_ledger=True)
        for plan in ((F.KERNEL_TBLOCK, 16, 16), (F.KERNEL_TBLOCK, 16, 64)):
            q, inv = gpu_run(prob, q0=q0, steps=steps, plan=plan)
            assert np.array_equal(q, ref), (steps, plan)
            assert inv["ledger"][0] == led


def test_wide_tiles_refused_outside_64_bit_direct_upwind():
    for flux, itype, lut in ((F.FLUX_BURGERS_EO, F.I64, False), (F.FLUX_UPWIND, F.I64, True)):
        u0, prob = make_case(flux, F.BC_PERIODIC, itype, 1000, seed=5, lut=lut)
        h = F.fqnm_create_from_field(prob, u0)
        try:
            with pytest.raises(F.FqnmError) as e:
                F.fqnm_set_plan(h, F.KERNEL_TBLOCK, 16, 40)
            assert e.value.status == F.ERR_ARG
        finally:
            F.fqnm_destroy(h)


def test_quantise_entry_point_matches_oracle():
    rng = np.random.default_rng(17)
    u = np.concatenate([rng.normal(0, 3, 100003), np.array([2.5, -3.5, 0.5]) * 1e-5])
    for itype, width in ((F.I32, 32), (F.I64, 64)):
        got = F.fqnm_quantise(u, 1e-5, itype).astype(np.int64)
        assert np.array_equal(got, O.quantise(u, 1e-5, width))
    with pytest.raises(F.FqnmError) as e:
        F.fqnm_quantise(np.array([1e10]), 1e-5, F.I32)
    assert e.value.status == F.ERR_RANGE
