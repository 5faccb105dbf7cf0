"""GPU parity of d-dimensional directional composition (Thm dimension_extension)
against the oracle's d-D stepper: integer states bit for bit, outflow ledgers
exactly.  Grids span several strips of the marching kernel along axis 0 with a
ragged tail, several row blocks along the marching axis with a ragged tail,
rows whose byte length is not a multiple of 16 (element loads), strips wider
than the grid, and single rows or columns."""
import numpy as np
import pytest

import oracle as O
from paper_2604_06947_amd import fqnm as F
from paper_2604_06947_amd import plans
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.gpu

KIND = {F.FLUX_UPWIND: O.UPWIND, F.FLUX_BURGERS_EO: O.BURGERS_EO,
        F.FLUX_BURGERS_GODUNOV: O.BURGERS_GODUNOV, F.FLUX_BURGERS_MURMAN_ROE: O.BURGERS_MURMAN_ROE,
        F.FLUX_LF_LINEAR: O.LF_LINEAR, F.FLUX_LF_BURGERS: O.LF_BURGERS}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    F.lib()


def axes_for(flux, shape, itype, bcs, lams, a_s=None, alphas=None, delta=1e-3):
    """fqnm_problem per direction; shape is the numpy shape (last axis contiguous)."""
    dim = len(shape)
    a_s = a_s or [1.0] * dim
    alphas = alphas or [0.0] * dim
    ext = shape[::-1]
    return [F.make_problem(flux, delta, lams[m], ext[m], bc=bcs[m], itype=itype, a=a_s[m],
                           alpha=alphas[m]) for m in range(dim)]


def oracle_axes(axes):
    return [O.Problem(KIND[p.flux], p.delta, p.lambda_, bc=p.bc,
                      width=32 if p.itype == F.I32 else 64, a=p.a, alpha=p.alpha) for p in axes]


def gpu_nd(axes, q0, steps, plan=None):
    h = F.fqnm_create_nd(axes, q0)
    try:
        if plan is not None:  # (vec, rows) of the marching kernel, or (kernel, vec, depth)
            F.fqnm_set_plan(h, *((F.KERNEL_ND_MARCH,) + tuple(plan) if len(plan) == 2 else plan))
        F.fqnm_step(h, steps)
        flat = F.fqnm_get_state(h, F.make_problem(axes[0].flux, axes[0].delta, axes[0].lambda_,
                                                  int(np.prod(q0.shape)), itype=axes[0].itype))
        inv = F.fqnm_invariants_get(h)
    finally:
        F.fqnm_destroy(h)
    return flat.astype(np.int64).reshape(q0.shape), inv


def field_q(shape, delta, seed, amp=1.0):
    rng = np.random.default_rng(seed)
    nd = len(shape)
    grids = np.meshgrid(*[np.arange(s) / s for s in shape], indexing="ij")
    u = 0.4 + amp * np.sin(2 * np.pi * grids[-1]) * np.cos(2 * np.pi * grids[0])
    if nd == 3:
        u = u + 0.3 * np.sin(2 * np.pi * grids[1])
    u = u + 0.5 * (grids[-1] >= rng.uniform(0.2, 0.8))
    return O.quantise(u.ravel(), delta).reshape(shape), float(np.max(np.abs(u)))


FLUXES = [(F.FLUX_UPWIND, [1.0, -0.7]), (F.FLUX_BURGERS_EO, None), (F.FLUX_BURGERS_GODUNOV, None),
          (F.FLUX_BURGERS_MURMAN_ROE, None), (F.FLUX_LF_LINEAR, [0.6, -0.4]),
          (F.FLUX_LF_BURGERS, None)]


def lams_for(flux, umax, a_s, dim):
    if flux == F.FLUX_UPWIND:
        return [0.9 / (dim * abs(a)) for a in a_s], None
    if flux == F.FLUX_LF_LINEAR:
        al = [1.2 * abs(a) for a in a_s]
        return [0.9 / (dim * x) for x in al], al
    if flux == F.FLUX_LF_BURGERS:
        al = [1.2 * umax] * dim
        return [0.9 / (dim * x) for x in al], al
    return [0.9 / (dim * umax)] * dim, None


@pytest.mark.parametrize("flux,a_s", FLUXES)
@pytest.mark.parametrize("itype", [F.I32, F.I64])
@pytest.mark.parametrize("bcs", [(F.BC_PERIODIC, F.BC_PERIODIC), (F.BC_OUTFLOW, F.BC_OUTFLOW),
                                 (F.BC_OUTFLOW, F.BC_PERIODIC)])
def test_nd_2d_matches_oracle(flux, a_s, itype, bcs):
    shape = (45, 602)  # (ny, nx): 2 strips + a tail at V=4 int32; rows 8-byte but not 16-byte aligned
    q0, umax = field_q(shape, 1e-3, seed=flux)
    a_s = a_s or [1.0, 1.0]
    lams, alphas = lams_for(flux, umax, a_s, 2)
    axes = axes_for(flux, shape, itype, bcs, lams, a_s, alphas)
    steps = 25
    ref, led = O.step_nd(oracle_axes(axes), q0, steps, return_ledger=True)
    plans = [(4, 16), (8, 7), (2, 9)] if itype == F.I32 else [(2, 16), (4, 5)]
    for plan in plans:
        got, inv = gpu_nd(axes, q0, steps, plan)
        assert np.array_equal(got, ref), plan
        assert inv["ledger"][0] == led, plan
        assert inv["sum"][0] == int(q0.sum()) + led


@pytest.mark.parametrize("flux,a_s", [(F.FLUX_UPWIND, [0.5, -1.0, 0.8]),
                                      (F.FLUX_BURGERS_EO, None), (F.FLUX_BURGERS_GODUNOV, None),
                                      (F.FLUX_LF_BURGERS, None)])
@pytest.mark.parametrize("itype", [F.I32, F.I64])
def test_nd_3d_matches_oracle(flux, a_s, itype):
    shape = (9, 6, 270)  # (nz, ny, nx)
    q0, umax = field_q(shape, 1e-3, seed=30 + flux)
    a_s = a_s or [1.0, 1.0, 1.0]
    lams, alphas = lams_for(flux, umax, a_s, 3)
    bcs = (F.BC_PERIODIC, F.BC_OUTFLOW, F.BC_OUTFLOW)
    axes = axes_for(flux, shape, itype, bcs, lams, a_s, alphas)
    steps = 12
    ref, led = O.step_nd(oracle_axes(axes), q0, steps, return_ledger=True)
    plans = [(4, 4), (8, 16)] if itype == F.I32 else [(2, 3), (4, 16)]
    for plan in plans:
        got, inv = gpu_nd(axes, q0, steps, plan)
        assert np.array_equal(got, ref), plan
        assert inv["ledger"][0] == led, plan


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (37, 1), (3, 5), (17, 301), (130, 9),
                                   (2, 3, 4), (1, 1, 77), (5, 1, 1)])
@pytest.mark.parametrize("bc", [F.BC_PERIODIC, F.BC_OUTFLOW])
def test_nd_small_and_ragged(shape, bc):
    q0, umax = field_q(shape, 1e-3, seed=len(shape) * 100 + shape[-1])
    dim = len(shape)
    axes = axes_for(F.FLUX_BURGERS_EO, shape, F.I32, [bc] * dim, [0.9 / (dim * umax)] * dim)
    ref, led = O.step_nd(oracle_axes(axes), q0, 9, return_ledger=True)
    for plan in [(4, 1), (8, 3), (2, 2)]:
        got, inv = gpu_nd(axes, q0, 9, plan)
        assert np.array_equal(got, ref), plan
        assert inv["ledger"][0] == led


def test_nd_counterexample_on_device():
    # the hand-worked loss of the maximum principle (two rounding steps adding up)
    q0 = np.zeros((4, 4), dtype=np.int64)
    q0[1, 1] = 3
    axes = axes_for(F.FLUX_UPWIND, q0.shape, F.I32, [F.BC_PERIODIC] * 2, [0.5, 0.5])
    got, _ = gpu_nd(axes, q0, 1)
    assert got[1, 1] == -1 and got.sum() == 3


def test_nd_refusals():
    q0 = np.zeros((8, 8), dtype=np.int32)
    ax = axes_for(F.FLUX_BURGERS_EO, q0.shape, F.I32, [F.BC_PERIODIC] * 2, [0.5, 0.5])
    ax[0].eval = F.EVAL_LUT
    with pytest.raises(F.FqnmError) as e:
        F.fqnm_create_nd(ax, q0)
    assert e.value.status == F.ERR_UNSUPPORTED
    # each direction within CFL 1, the sum above it
    q0 = np.full((8, 8), 1000, dtype=np.int32)  # u = 1 at delta 1e-3
    ax = axes_for(F.FLUX_BURGERS_EO, q0.shape, F.I32, [F.BC_PERIODIC] * 2, [0.6, 0.6])
    with pytest.raises(F.FqnmError) as e:
        F.fqnm_create_nd(ax, q0)
    assert e.value.status == F.ERR_CFL
    ax = axes_for(F.FLUX_BURGERS_EO, q0.shape, F.I32, [F.BC_PERIODIC] * 2, [0.3, 0.3])
    ax[1].delta = 2e-3
    with pytest.raises(F.FqnmError) as e:
        F.fqnm_create_nd(ax, q0)
    assert e.value.status == F.ERR_ARG


def test_nd_levels_and_autotune():
    shape = (33, 520)
    q0, umax = field_q(shape, 1e-3, seed=77)
    axes = axes_for(F.FLUX_BURGERS_GODUNOV, shape, F.I32, [F.BC_PERIODIC] * 2,
                    [0.4 / umax, 0.4 / umax])
    oax = oracle_axes(axes)
    h = F.fqnm_create_nd(axes, q0)
    try:
        F.fqnm_autotune(h, 8)
        F.fqnm_step(h, 10)
        ref = O.step_nd(oax, q0, 10)
        S, _ = F.fqnm_entropy(h)
        assert S == O.entropy(ref.ravel())
        f, t, c, rho = F.fqnm_step_transitions(h, ref.size)
        ref1 = O.step_nd(oax, ref, 1)
        f0, t0, c0 = O.level_transitions(ref.ravel(), ref1.ravel())
        assert np.array_equal(f, f0) and np.array_equal(t, t0) and np.array_equal(c, c0)
        assert rho == O.row_defect(ref.ravel(), ref1.ravel())
    finally:
        F.fqnm_destroy(h)


W6_PLANS = {"default": None,
            "benchmarked": (plans.ND_PLAN_W6[0], plans.ND_PLAN_W6[1],
                            F.nd_tb_depth(plans.ND_PLAN_W6[2], plans.ND_PLAN_W6[3])),
            "one_step": plans.ND_MARCH_PLAN_W6}


@pytest.mark.parametrize("plan", list(W6_PLANS))
def test_nd_w6_full_size_sampled(plan):
    """W6 at its full 4096 x 4096 cells, 40 steps on the device (with the
    default plan, the benchmarked one and one step per launch); cells sampled
    and checked against the oracle run on the (2s+1)^2 window around each (the
    5-point composition reaches s cells per direction in s steps)."""
    w = W.w6_burgers_2d()
    ny, nx = w.shape
    q0 = O.quantise(w.u0.ravel(), w.delta, 32).reshape(w.shape)
    axes = axes_for(F.FLUX_BURGERS_EO, w.shape, F.I32, [F.BC_PERIODIC] * 2, list(w.lam),
                    delta=w.delta)
    s = 40
    got, inv = gpu_nd(axes, q0, s, W6_PLANS[plan])
    assert inv["sum"][0] == int(q0.sum())
    oax = [O.Problem(O.BURGERS_EO, w.delta, w.lam[m], bc=O.OUTFLOW, width=32) for m in range(2)]
    rng = np.random.default_rng(66)
    pts = [(0, 0), (ny - 1, nx - 1), (ny // 2, int(w.u0[0].argmax()))]
    pts += [(int(a), int(b)) for a, b in zip(rng.integers(0, ny, 5), rng.integers(0, nx, 5))]
    for (j, i) in pts:
        jj = np.arange(j - s, j + s + 1) % ny
        ii = np.arange(i - s, i + s + 1) % nx
        win = q0[np.ix_(jj, ii)]
        ref = O.step_nd(oax, win, s)
        assert got[j, i] == ref[s, s], (j, i)


# ---------------------------------------------------------------------------
# Temporal blocking on 2-D periodic int32 grids (kernel 9)
# ---------------------------------------------------------------------------
TB_PERIODIC = (F.BC_PERIODIC, F.BC_PERIODIC)


def tb_case(flux, a_s, shape, seed, same=True, itype=F.I32, bcs=TB_PERIODIC):
    q0, umax = field_q(shape, 1e-3, seed=seed)
    a_s = a_s or [1.0, 1.0]
    lams, alphas = lams_for(flux, umax, a_s, 2)
    if not same:  # different constants per axis: the marching axis evaluates its own maps
        lams = [lams[0], 0.8 * lams[1]]
    return q0, axes_for(flux, shape, itype, bcs, lams, a_s, alphas)


TB_PLANS = {F.I32: [(4, 4, 0), (4, 8, 16), (2, 2, 7), (2, 8, 3), (4, 1, 5), (2, 4, 64)],
            F.I64: [(2, 4, 0), (2, 8, 16), (2, 2, 7), (2, 1, 3)]}


@pytest.mark.parametrize("flux,a_s", FLUXES)
@pytest.mark.parametrize("same", [True, False])
@pytest.mark.parametrize("itype", [F.I32, F.I64])
def test_nd_tb_matches_oracle(flux, a_s, same, itype):
    # 45 rows x 604 cells: several strips with a ragged last one at every
    # (vec, depth), row blocks with a ragged tail; 13 steps = passes of 8, 4, 1
    shape = (45, 604)
    q0, axes = tb_case(flux, a_s, shape, seed=200 + flux, same=same, itype=itype)
    steps = 13
    ref, led = O.step_nd(oracle_axes(axes), q0, steps, return_ledger=True)
    assert led == 0
    for vec, K, rows in TB_PLANS[itype]:
        got, inv = gpu_nd(axes, q0, steps, (F.KERNEL_ND_TB, vec, F.nd_tb_depth(K, rows)))
        assert np.array_equal(got, ref), (vec, K, rows)
        assert inv["ledger"][0] == 0 and inv["sum"][0] == int(q0.sum())


@pytest.mark.parametrize("shape", [(1, 4), (2, 8), (7, 4), (3, 260), (130, 12), (9, 1000),
                                   (64, 256)])
@pytest.mark.parametrize("bc", [F.BC_PERIODIC, F.BC_OUTFLOW])
def test_nd_tb_small_and_ragged(shape, bc):
    # grids narrower than one strip (cells wrap or clamp inside a wavefront),
    # fewer rows than the steps per pass, single rows
    q0, axes = tb_case(F.FLUX_BURGERS_EO, None, shape, seed=shape[0] * 1000 + shape[1],
                       bcs=(bc, bc))
    ref, led = O.step_nd(oracle_axes(axes), q0, 11, return_ledger=True)
    for vec, K, rows in [(4, 8, 0), (2, 4, 1), (4, 2, 3), (2, 1, 2)]:
        got, inv = gpu_nd(axes, q0, 11, (F.KERNEL_ND_TB, vec, F.nd_tb_depth(K, rows)))
        assert np.array_equal(got, ref), (vec, K, rows)
        assert inv["ledger"][0] == led, (vec, K, rows)


@pytest.mark.parametrize("flux,a_s", FLUXES)
@pytest.mark.parametrize("bcs", [(F.BC_OUTFLOW, F.BC_OUTFLOW), (F.BC_OUTFLOW, F.BC_PERIODIC),
                                 (F.BC_PERIODIC, F.BC_OUTFLOW)])
@pytest.mark.parametrize("itype", [F.I32, F.I64])
def test_nd_tb_outflow_matches_oracle(flux, a_s, bcs, itype):
    # outflow ends on either axis: states and the boundary ledger, with strips
    # and row blocks that end on the grid's edges and inside it
    shape = (45, 604)
    q0, axes = tb_case(flux, a_s, shape, seed=300 + flux, itype=itype, bcs=bcs)
    steps = 13
    ref, led = O.step_nd(oracle_axes(axes), q0, steps, return_ledger=True)
    for vec, K, rows in TB_PLANS[itype]:
        got, inv = gpu_nd(axes, q0, steps, (F.KERNEL_ND_TB, vec, F.nd_tb_depth(K, rows)))
        assert np.array_equal(got, ref), (vec, K, rows)
        assert inv["ledger"][0] == led, (vec, K, rows)
        assert inv["sum"][0] == int(q0.sum()) + led


def test_nd_tb_refusals():
    q0 = np.zeros((8, 8), dtype=np.int32)
    ok = axes_for(F.FLUX_BURGERS_EO, q0.shape, F.I32, TB_PERIODIC, [0.3, 0.3])
    bad = [axes_for(F.FLUX_BURGERS_EO, q0.shape, F.I64, TB_PERIODIC, [0.3, 0.3])]  # vec 4
    for ax in bad:
        h = F.fqnm_create_nd(ax, q0)
        try:
            with pytest.raises(F.FqnmError) as e:
                F.fqnm_set_plan(h, F.KERNEL_ND_TB, 4, F.nd_tb_depth(4))
            assert e.value.status == F.ERR_ARG
        finally:
            F.fqnm_destroy(h)
    q3 = np.zeros((4, 4, 8), dtype=np.int32)
    h = F.fqnm_create_nd(axes_for(F.FLUX_BURGERS_EO, q3.shape, F.I32, [F.BC_PERIODIC] * 3,
                                  [0.2] * 3), q3)
    try:
        with pytest.raises(F.FqnmError):
            F.fqnm_set_plan(h, F.KERNEL_ND_TB, 4, F.nd_tb_depth(4))
    finally:
        F.fqnm_destroy(h)
    q6 = np.zeros((8, 6), dtype=np.int32)  # axis 0 of 6 cells: not a multiple of 4
    h = F.fqnm_create_nd(axes_for(F.FLUX_BURGERS_EO, q6.shape, F.I32, TB_PERIODIC, [0.3, 0.3]), q6)
    try:
        with pytest.raises(F.FqnmError):
            F.fqnm_set_plan(h, F.KERNEL_ND_TB, 4, F.nd_tb_depth(4))
        F.fqnm_set_plan(h, F.KERNEL_ND_TB, 2, F.nd_tb_depth(4))  # 6 is a multiple of 2
    finally:
        F.fqnm_destroy(h)
    h = F.fqnm_create_nd(ok, q0)
    try:
        for K in (3, 5, 16):
            with pytest.raises(F.FqnmError):
                F.fqnm_set_plan(h, F.KERNEL_ND_TB, 4, F.nd_tb_depth(K))
    finally:
        F.fqnm_destroy(h)


def test_nd_tb_autotune_and_levels():
    shape = (40, 520)
    q0, axes = tb_case(F.FLUX_BURGERS_GODUNOV, None, shape, seed=91)
    oax = oracle_axes(axes)
    h = F.fqnm_create_nd(axes, q0)
    try:
        F.fqnm_autotune(h, 8)
        assert F.fqnm_get_plan(h)["kernel"] in (F.KERNEL_ND_MARCH, F.KERNEL_ND_TB)
        for kernel, vec, depth in [(F.KERNEL_ND_TB, 4, F.nd_tb_depth(8, 4)), (0, 0, 0)]:
            if kernel:
                F.fqnm_set_plan(h, kernel, vec, depth)
            F.fqnm_step(h, 9)
        ref = O.step_nd(oax, q0, 18)
        flat = F.fqnm_get_state(h, F.make_problem(axes[0].flux, axes[0].delta, axes[0].lambda_,
                                                  q0.size, itype=F.I32))
        assert np.array_equal(flat.astype(np.int64).reshape(shape), ref)
    finally:
        F.fqnm_destroy(h)


def test_nd_tuned_plan_not_reused_across_boundary_kinds():
    # a plan tuned (or set) on a periodic grid is cached for that grid's key;
    # an outflow grid of the same extents and kind must not pick it up
    shape = (24, 264)
    q0, axes = tb_case(F.FLUX_BURGERS_EO, None, shape, seed=123)
    h = F.fqnm_create_nd(axes, q0)
    try:
        assert F.fqnm_get_plan(h)["kernel"] == F.KERNEL_ND_TB  # the default of such grids
        F.fqnm_autotune(h, 8)
    finally:
        F.fqnm_destroy(h)
    out_axes = axes_for(F.FLUX_BURGERS_EO, shape, F.I32, (F.BC_OUTFLOW, F.BC_OUTFLOW),
                        [a.lambda_ for a in axes])
    ref, led = O.step_nd(oracle_axes(out_axes), q0, 9, return_ledger=True)
    h = F.fqnm_create_nd(out_axes, q0)
    try:
        assert F.fqnm_get_plan(h)["kernel"] in (F.KERNEL_ND_MARCH, F.KERNEL_ND_TB)
        F.fqnm_step(h, 9)
        flat = F.fqnm_get_state(h, F.make_problem(F.FLUX_BURGERS_EO, axes[0].delta,
                                                  axes[0].lambda_, q0.size, itype=F.I32))
        inv = F.fqnm_invariants_get(h)
    finally:
        F.fqnm_destroy(h)
    assert np.array_equal(flat.astype(np.int64).reshape(shape), ref)
    assert inv["ledger"][0] == led


def test_nd_plan_switch_takes_defaults():
    q0, axes = tb_case(F.FLUX_BURGERS_EO, None, (16, 128), seed=5)
    h = F.fqnm_create_nd(axes, q0)
    try:
        F.fqnm_set_plan(h, F.KERNEL_ND_TB, 4, F.nd_tb_depth(8, 24))
        F.fqnm_set_plan(h, F.KERNEL_ND_MARCH)
        pl = F.fqnm_get_plan(h)
        assert (pl["kernel"], pl["vec"], pl["depth"]) == (F.KERNEL_ND_MARCH, 4, 16)
        F.fqnm_set_plan(h, F.KERNEL_ND_TB)
        pl = F.fqnm_get_plan(h)
        assert (pl["kernel"], pl["vec"], pl["depth"]) == (F.KERNEL_ND_TB, 2, 4)
        F.fqnm_step(h, 6)
        flat = F.fqnm_get_state(h, F.make_problem(axes[0].flux, axes[0].delta, axes[0].lambda_,
                                                  q0.size, itype=F.I32))
    finally:
        F.fqnm_destroy(h)
    ref = O.step_nd(oracle_axes(axes), q0, 6)
    assert np.array_equal(flat.astype(np.int64).reshape(q0.shape), ref)


@pytest.mark.parametrize("flux", [F.FLUX_BURGERS_EO, F.FLUX_BURGERS_GODUNOV])
@pytest.mark.parametrize("bcs", [(F.BC_OUTFLOW, F.BC_OUTFLOW), (F.BC_OUTFLOW, F.BC_PERIODIC),
                                 (F.BC_PERIODIC, F.BC_OUTFLOW)])
@pytest.mark.parametrize("itype", [F.I32, F.I64])
def test_nd_tb_halo_past_an_outflow_end(flux, bcs, itype):
    # 602 cells along axis 0: with 2 cells per lane and 4 steps per pass the
    # strip storing cells 480..599 loads cells up to 603, past the end, though
    # none of its stored cells is an end cell; with 12 rows per wavefront the
    # block storing rows 24..35 loads rows past the last row (36) likewise
    shape = (37, 602)
    q0, axes = tb_case(flux, None, shape, seed=602 + flux, itype=itype, bcs=bcs)
    steps = 15
    ref, led = O.step_nd(oracle_axes(axes), q0, steps, return_ledger=True)
    for vec, K, rows in [(2, 4, 12), (2, 8, 16), (2, 2, 5), (2, 1, 7)]:
        got, inv = gpu_nd(axes, q0, steps, (F.KERNEL_ND_TB, vec, F.nd_tb_depth(K, rows)))
        assert np.array_equal(got, ref), (vec, K, rows)
        assert inv["ledger"][0] == led, (vec, K, rows)


def test_nd_default_plans():
    # 2-D grids start on the temporally blocked kernel, or on the one-step
    # kernel when axis 0 has an odd length; both give the oracle's integers
    for shape, kernel in [((20, 64), F.KERNEL_ND_TB), ((20, 37), F.KERNEL_ND_MARCH)]:
        q0, axes = tb_case(F.FLUX_BURGERS_EO, None, shape, seed=shape[1])
        h = F.fqnm_create_nd(axes, q0)
        try:
            assert F.fqnm_get_plan(h)["kernel"] == kernel, shape
        finally:
            F.fqnm_destroy(h)
        got, _ = gpu_nd(axes, q0, 10)
        assert np.array_equal(got, O.step_nd(oracle_axes(axes), q0, 10)), shape
