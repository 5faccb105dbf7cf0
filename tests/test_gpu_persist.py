"""Persistent temporal blocking (plan kernel 10): every pass of a temporally
blocked plan in one cooperative launch, tiles handing their edge cells to
their neighbours through memory between passes.  Bit-exact against the
oracle on grids of one, two and many tiles, ragged sizes, step counts that
are not a multiple of the depth, repeated calls on one context (the pass
tags continue), table and direct evaluation; plans it does not cover are
refused."""
import numpy as np
import pytest

import oracle as O
from paper_2604_06947_amd import fqnm as F
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.gpu
KERNEL_PERSIST = 10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    F.lib()


def burgers(n, lut, seed=2):
    w = W.w2_burgers_step(n=n, steps=1, seed=seed)
    prob = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam, n, itype=F.I32,
                          eval_=F.EVAL_LUT if lut else F.EVAL_DIRECT)
    op = O.Problem(O.BURGERS_EO, w.delta, w.lam, width=32)
    return O.quantise(w.u0, w.delta, 32), prob, op


@pytest.mark.parametrize("n,vec,depth,steps", [
    (200, 4, 8, 30), (400, 4, 8, 50), (1000, 4, 8, 37), (5003, 4, 40, 150),
    (2113, 4, 24, 100), (44033, 8, 64, 130), (300001, 4, 40, 400), (300001, 4, 16, 123)])
@pytest.mark.parametrize("lut", [True, False])
def test_persistent_plan_matches_oracle(n, vec, depth, steps, lut):
    q0, prob, op = burgers(n, lut)
    print("persist", n, vec, depth, steps, lut, flush=True)
    h = F.fqnm_create(prob, q0.astype(np.int32))
    try:
        F.fqnm_set_plan(h, KERNEL_PERSIST, vec, depth)
        F.fqnm_step(h, steps)
        got = F.fqnm_get_state(h, prob).astype(np.int64)
        assert np.array_equal(got, O.step(op, q0, steps))
        F.fqnm_step(h, 3 * depth + 1)  # a second launch on the same exchange buffer
        got = F.fqnm_get_state(h, prob).astype(np.int64)
        assert np.array_equal(got, O.step(op, q0, steps + 3 * depth + 1))
        inv = F.fqnm_invariants_get(h)
        assert inv["sum"][0] == int(q0.sum())
    finally:
        F.fqnm_destroy(h)


def test_persistent_upwind_and_w1():
    w = W.w1_advection_square()
    prob = F.make_problem(F.FLUX_UPWIND, w.delta, w.lam, w.n, itype=F.I32, a=w.a)
    op = O.Problem(O.UPWIND, w.delta, w.lam, width=32, a=w.a)
    q0 = O.quantise(w.u0, w.delta, 32)
    for lut in (False, True):
        prob.eval = F.EVAL_LUT if lut else F.EVAL_DIRECT
        h = F.fqnm_create(prob, q0.astype(np.int32))
        try:
            F.fqnm_set_plan(h, KERNEL_PERSIST, 4, 24)
            F.fqnm_step(h, w.steps)
            assert np.array_equal(F.fqnm_get_state(h, prob).astype(np.int64),
                                  O.step(op, q0, w.steps))
        finally:
            F.fqnm_destroy(h)


def test_persistent_plan_refused_where_it_does_not_apply():
    q0, prob, op = burgers(5000, True)
    prob.bc = F.BC_OUTFLOW
    h = F.fqnm_create(prob, q0.astype(np.int32))
    try:
        with pytest.raises(F.FqnmError):
            F.fqnm_set_plan(h, KERNEL_PERSIST, 4, 40)
    finally:
        F.fqnm_destroy(h)
    prob.bc = F.BC_PERIODIC
    h = F.fqnm_create(prob, q0.astype(np.int32))
    try:
        with pytest.raises(F.FqnmError):  # tiles shorter than the halo
            F.fqnm_set_plan(h, KERNEL_PERSIST, 4, 100)
        with pytest.raises(F.FqnmError):
            F.fqnm_set_plan(h, KERNEL_PERSIST, 16, 40)
    finally:
        F.fqnm_destroy(h)
    p64 = F.make_problem(F.FLUX_BURGERS_EO, prob.delta, prob.lambda_, 5000, itype=F.I64)
    h = F.fqnm_create(p64, q0)
    try:
        with pytest.raises(F.FqnmError):
            F.fqnm_set_plan(h, KERNEL_PERSIST, 4, 40)
    finally:
        F.fqnm_destroy(h)
