"""GPU parity of the componentwise quantised Roe transfer (Euler, 3 x int64)."""
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


def test_fp64_div_sqrt_match_host():
    """The Euler transfer needs correctly rounded FP64 division and square root
    on the device; numpy's are IEEE correctly rounded on the host."""
    import torch
    rng = np.random.default_rng(77)
    n = 4_000_000
    a = np.concatenate([
        rng.uniform(0, 4, n // 4), np.exp(rng.uniform(-700, 700, n // 4)),
        rng.uniform(1e-6, 1e-3, n // 4), rng.random(n // 4) * 2.0 ** rng.integers(-60, 60, n // 4),
        np.array([0.0, 1.0, 2.0, 4.0, 0.25, 1e-300, 5e-324, 1.7976931348623157e308,
                  2.0 ** -1022, 0.30313017805064685, 0.9274526200489499])])
    b = np.concatenate([rng.uniform(1e-3, 3, a.size - 11),
                        np.array([1.0, 3.0, 7.0, 0.1, 1e-300, 1e300, 2.0, 0.5, 3.0, 0.4, 1.4])])
    da, db = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
    ds, dd = torch.empty_like(da), torch.empty_like(da)
    F.fqnm_fp64_selfcheck(da.data_ptr(), db.data_ptr(), ds.data_ptr(), dd.data_ptr(), a.size,
                          torch.cuda.current_stream().cuda_stream)
    s, d = ds.cpu().numpy(), dd.cpu().numpy()
    assert np.array_equal(s.view(np.uint64), np.sqrt(a).view(np.uint64))
    with np.errstate(over="ignore"):  # exp(700) / 1e-3 overflows to inf on both sides
        ref = a / b
    assert np.array_equal(d.view(np.uint64), ref.view(np.uint64))


def euler_case(n, kind, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), bc=F.BC_OUTFLOW):
    r = W.sod_request(n, left, right, kind=kind)
    prob = F.make_problem(kind, r.delta, r.lam, n, bc=bc, itype=F.I64, gamma=r.gamma)
    op = O.Problem(kind, r.delta, r.lam, bc=bc, width=64, gamma=r.gamma)
    return r, prob, op


@pytest.mark.parametrize("kind", [F.FLUX_EULER_ROE, F.FLUX_EULER_ROE_EF])
@pytest.mark.parametrize("n", [1024, 777])
def test_sod_full_trajectory_bitexact(kind, n):
    r, prob, op = euler_case(n, kind)
    q0 = np.stack([O.quantise(r.U0[c], r.delta, 64) for c in range(3)])
    ref, led = O.step_euler(op, q0, r.steps, return_ledger=True)
    h = F.fqnm_create_from_field(prob, r.U0.ravel())
    try:
        assert np.array_equal(F.fqnm_get_state(h, prob), q0)
        F.fqnm_step(h, r.steps)
        q = F.fqnm_get_state(h, prob)
        inv = F.fqnm_invariants_get(h)
    finally:
        F.fqnm_destroy(h)
    assert np.array_equal(q, ref)
    assert inv["ledger"] == [int(v) for v in led]
    assert inv["sum"] == [int(v) for v in ref.sum(axis=1)]


def test_transonic_and_periodic_bitexact():
    for left, right, bc in [((1.0, 0.75, 1.0), (0.125, 0.0, 0.1), F.BC_OUTFLOW),
                            ((0.125, 0.0, 0.1), (1.0, -0.75, 1.0), F.BC_PERIODIC)]:
        r, prob, op = euler_case(600, F.FLUX_EULER_ROE_EF, left, right, bc)
        q0 = np.stack([O.quantise(r.U0[c], r.delta, 64) for c in range(3)])
        ref = O.step_euler(op, q0, 400)
        h = F.fqnm_create(prob, q0)
        try:
            F.fqnm_step(h, 400)
            q = F.fqnm_get_state(h, prob)
        finally:
            F.fqnm_destroy(h)
        assert np.array_equal(q, ref)


def test_tiny_euler_grids():
    for n in (1, 2, 3, 253, 254, 255, 509):
        r, prob, op = euler_case(max(n, 2) if n > 1 else 1, F.FLUX_EULER_ROE_EF)
        q0 = np.stack([O.quantise(r.U0[c], r.delta, 64) for c in range(3)])
        ref = O.step_euler(op, q0, 25)
        h = F.fqnm_create(prob, q0)
        try:
            F.fqnm_step(h, 25)
            q = F.fqnm_get_state(h, prob)
        finally:
            F.fqnm_destroy(h)
        assert np.array_equal(q, ref), n
