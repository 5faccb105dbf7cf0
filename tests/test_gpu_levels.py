"""GPU parity of the level statistics (Supplementary Information: eq:pk_definition,
eq:discrete_entropy, eq:neff, Definition level_transition, eq:empirical_M and the
row-sum defect) against the oracle.  Levels, counts and transition triples are
integers and must match exactly; S and the row-sum defect are summed in the
same order on both sides (increasing level), so they must match to the last bit
up to the host libm's log, which both sides share."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2604_06947_amd import fqnm as F
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.gpu

KIND = {F.FLUX_UPWIND: O.UPWIND, F.FLUX_BURGERS_EO: O.BURGERS_EO,
        F.FLUX_BURGERS_GODUNOV: O.BURGERS_GODUNOV, F.FLUX_LF_LINEAR: O.LF_LINEAR}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    F.lib()


def _oracle_problem(prob):
    return O.Problem(KIND[prob.flux], prob.delta, prob.lambda_, bc=prob.bc,
                     width=32 if prob.itype == F.I32 else 64, a=prob.a, alpha=prob.alpha)


def _check_state(prob, q0, steps_before=0):
    """Histogram and entropy after `steps_before` steps, then one transition step."""
    op = _oracle_problem(prob)
    q_ref = O.step(op, q0, steps_before) if steps_before else np.asarray(q0, np.int64)
    h = F.fqnm_create(prob, np.asarray(q0, F._np_itype(prob)))
    try:
        F.fqnm_step(h, steps_before)
        lv, ct = F.fqnm_level_histogram(h)
        lv_ref, ct_ref = O.level_histogram(q_ref)
        assert np.array_equal(lv, lv_ref) and np.array_equal(ct, ct_ref)
        S, neff = F.fqnm_entropy(h)
        S_ref = O.entropy(q_ref)
        assert S == S_ref, (S, S_ref)
        assert neff == math.exp(S_ref)
        f, t, c, rho = F.fqnm_step_transitions(h, prob.n)
        q_next = O.step(op, q_ref, 1)
        f_ref, t_ref, c_ref = O.level_transitions(q_ref, q_next)
        assert np.array_equal(f, f_ref) and np.array_equal(t, t_ref) and np.array_equal(c, c_ref)
        assert rho == O.row_defect(q_ref, q_next), (rho, O.row_defect(q_ref, q_next))
        # the transition step is an ordinary step of the context
        assert np.array_equal(F.fqnm_get_state(h, prob).astype(np.int64), q_next)
        assert F.fqnm_invariants_get(h)["steps_done"] == steps_before + 1
    finally:
        F.fqnm_destroy(h)


def test_levels_w1_advection():
    w = W.w1_advection_square()
    prob = F.make_problem(F.FLUX_UPWIND, w.delta, w.lam, w.n, itype=F.I32)
    q0 = O.quantise(w.u0, w.delta, 32)
    _check_state(prob, q0, steps_before=37)


@pytest.mark.parametrize("itype", [F.I32, F.I64])
@pytest.mark.parametrize("flux", [F.FLUX_BURGERS_EO, F.FLUX_BURGERS_GODUNOV])
def test_levels_burgers_shock(itype, flux):
    # a few thousand cells over several hundred levels, a shock forming
    w = W.w2_burgers_step(n=5003, steps=1)
    prob = F.make_problem(flux, 1e-3, w.lam, w.n, itype=itype)
    q0 = O.quantise(w.u0, 1e-3, 32 if itype == F.I32 else 64)
    _check_state(prob, q0, steps_before=900)


@pytest.mark.parametrize("lo,hi", [(-3, 4), (-200000, 200000), (-(1 << 50), 1 << 50)])
def test_levels_random_int64(lo, hi):
    # many levels with one cell each, and levels far from zero (sign handling of
    # the radix sort); LF with alpha covering the range keeps CFL valid
    n = 4099
    q0 = W.random_states(n, lo, hi, seed=71)
    umax = max(abs(lo), abs(hi)) * 1e-6
    prob = F.make_problem(F.FLUX_LF_LINEAR, 1e-6, 0.5 / max(umax, 1.0), n, itype=F.I64,
                          a=0.5, alpha=1.0)
    _check_state(prob, q0)


@pytest.mark.parametrize("lo,hi", [(-150000, 150000), (-(1 << 20), 1 << 20),
                                   (-(1 << 40), 1 << 40)])
def test_levels_random_int64_many_tiles(lo, hi):
    # the first range is counted directly (at most 4n levels), each block
    # spanning far more levels than its LDS histogram holds; the others take
    # the sort: 73 tiles with a ragged last one, and for the widest range the
    # two-sort path for the transition pairs (their packed key needs 82 bits)
    n = 300007
    q0 = W.random_states(n, lo, hi, seed=72)
    umax = max(abs(lo), abs(hi)) * 1e-6
    prob = F.make_problem(F.FLUX_LF_LINEAR, 1e-6, 0.5 / max(umax, 1.0), n, itype=F.I64,
                          a=0.5, alpha=1.0)
    _check_state(prob, q0)


def test_levels_constant_and_tiny():
    for n, val in [(1, 5), (2, -7), (64, 0), (1000, 123456)]:
        prob = F.make_problem(F.FLUX_UPWIND, 1e-3, 0.5, n, itype=F.I32)
        q0 = np.full(n, val, np.int64)
        _check_state(prob, q0)
        h = F.fqnm_create(prob, q0.astype(np.int32))
        try:
            assert F.fqnm_entropy(h) == (0.0, 1.0)
        finally:
            F.fqnm_destroy(h)


def test_levels_partial_capacity():
    n = 777
    q0 = W.random_states(n, -50, 50, seed=3)
    prob = F.make_problem(F.FLUX_UPWIND, 1e-3, 0.5, n, itype=F.I32)
    lv_ref, ct_ref = O.level_histogram(q0)
    h = F.fqnm_create(prob, q0.astype(np.int32))
    try:
        import ctypes as C
        m = C.c_int64(0)
        lv = np.zeros(10, np.int64)
        ct = np.zeros(10, np.int64)
        F._check(F.lib().fqnm_level_histogram(h, lv.ctypes.data, ct.ctypes.data, 10, C.byref(m)))
        assert m.value == lv_ref.size
        assert np.array_equal(lv, lv_ref[:10]) and np.array_equal(ct, ct_ref[:10])
    finally:
        F.fqnm_destroy(h)


def test_levels_full_size_w2_first_step():
    """W2 at its full 2^20 cells: histogram, entropy and the transitions of the
    first step against the oracle (one oracle step of 2^20 cells)."""
    w = W.w2_burgers_step()
    prob = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam, w.n, itype=F.I32,
                          eval_=F.EVAL_LUT)
    q0 = O.quantise(w.u0, w.delta, 32)
    _check_state(prob, q0)


def test_levels_refuse_other_contexts():
    req = W.sod_request(256)
    prob = F.make_problem(F.FLUX_EULER_ROE_EF, req.delta, req.lam, req.n, bc=F.BC_OUTFLOW,
                          itype=F.I64, gamma=1.4)
    h = F.fqnm_create_from_field(prob, req.U0.ravel())
    try:
        with pytest.raises(F.FqnmError) as e:
            F.fqnm_entropy(h)
        assert e.value.status == F.ERR_UNSUPPORTED
    finally:
        F.fqnm_destroy(h)
    u0 = W.random_smooth_step(512, seed=1, b=0.1)
    prob = F.make_problem(F.FLUX_BURGERS_EO, 1e-5, 0.4, 512)
    h = F.fqnm_create_classical(prob, u0)
    try:
        with pytest.raises(F.FqnmError) as e:
            F.fqnm_level_histogram(h)
        assert e.value.status == F.ERR_UNSUPPORTED
    finally:
        F.fqnm_destroy(h)
