"""GPU parity of the density-only quantised Roe update (Sec. 3.3, the paper's
prototype) against the oracle: density counts bit for bit, and the FP64
momentum and energy bit for bit as well (both sides run the same IEEE
operations in the same order, compiled without contraction)."""
import numpy as np
import pytest

import oracle as O
from paper_2604_06947_amd import fqnm as F
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.gpu

KIND = {F.FLUX_EULER_ROE_DENSITY: O.EULER_ROE, F.FLUX_EULER_ROE_EF_DENSITY: O.EULER_ROE_EF}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    F.lib()


def case(n, kind, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), bc=F.BC_OUTFLOW):
    r = W.sod_request(n, left, right, kind=KIND[kind])
    prob = F.make_problem(kind, r.delta, r.lam, n, bc=bc, itype=F.I64, gamma=r.gamma)
    op = O.Problem(KIND[kind], r.delta, r.lam, bc=bc, width=64, gamma=r.gamma)
    qr = O.quantise(r.U0[0], r.delta, 64)
    return r, prob, op, (qr, r.U0[1].copy(), r.U0[2].copy())


def same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float64).view(np.uint64),
                          np.asarray(b, np.float64).view(np.uint64))


@pytest.mark.parametrize("kind", [F.FLUX_EULER_ROE_DENSITY, F.FLUX_EULER_ROE_EF_DENSITY])
@pytest.mark.parametrize("n", [1024, 777, 255, 256, 3])
def test_density_only_sod_matches_oracle(kind, n):
    r, prob, op, st0 = case(n, kind)
    qr, m, E, led = O.step_euler_density(op, *st0, r.steps, return_ledger=True)
    h = F.fqnm_create_from_field(prob, r.U0.ravel())
    try:
        g0 = F.density_only_state(F.fqnm_get_state(h, prob))
        assert np.array_equal(g0[0], st0[0]) and same_bits(g0[1], st0[1])
        F.fqnm_step(h, r.steps)
        gq, gm, gE = F.density_only_state(F.fqnm_get_state(h, prob))
        inv = F.fqnm_invariants_get(h)
        u = F.fqnm_reconstruct(h, prob)
    finally:
        F.fqnm_destroy(h)
    assert np.array_equal(gq, qr)
    assert same_bits(gm, m) and same_bits(gE, E)
    assert inv["components"] == 1 and inv["ledger"][0] == led
    assert inv["sum"][0] == int(st0[0].sum()) + led
    assert same_bits(u[0], O.reconstruct(qr, r.delta)) and same_bits(u[1], m)


def test_density_only_periodic_jittered_from_raw_state():
    rng = np.random.default_rng(12)
    n = 2000
    r, prob, op, (qr, m, E) = case(n, F.FLUX_EULER_ROE_EF_DENSITY, bc=F.BC_PERIODIC)
    x = W.grid(n)
    qr = O.quantise(0.6 + 0.3 * np.sin(2 * np.pi * x) + 0.05 * rng.random(n), r.delta, 64)
    m = 0.2 * np.cos(2 * np.pi * x)
    E = 1.5 + 0.2 * rng.random(n)
    ref = O.step_euler_density(op, qr, m, E, 300)
    h = F.fqnm_create(prob, F.density_only_raw(qr, m, E))
    try:
        F.fqnm_step(h, 300)
        got = F.density_only_state(F.fqnm_get_state(h, prob))
        inv = F.fqnm_invariants_get(h)
    finally:
        F.fqnm_destroy(h)
    assert np.array_equal(got[0], ref[0]) and same_bits(got[1], ref[1]) and same_bits(got[2], ref[2])
    assert inv["sum"][0] == int(qr.sum())


def test_componentwise_unchanged_next_to_density_only():
    # the componentwise kind runs through the same kernel with the flag off
    r = W.sod_request(512, kind=O.EULER_ROE_EF)
    prob = F.make_problem(F.FLUX_EULER_ROE_EF, r.delta, r.lam, 512, bc=F.BC_OUTFLOW, itype=F.I64,
                          gamma=r.gamma)
    op = O.Problem(O.EULER_ROE_EF, r.delta, r.lam, bc=O.OUTFLOW, width=64, gamma=r.gamma)
    q0 = np.stack([O.quantise(r.U0[c], r.delta, 64) for c in range(3)])
    ref = O.step_euler(op, q0, r.steps)
    h = F.fqnm_create_from_field(prob, r.U0.ravel())
    try:
        F.fqnm_step(h, r.steps)
        assert np.array_equal(F.fqnm_get_state(h, prob), ref)
    finally:
        F.fqnm_destroy(h)


def test_density_only_through_the_server():
    reqs = []
    for i, n in enumerate([64, 300, 1024, 2001]):
        kind = F.FLUX_EULER_ROE_DENSITY if i % 2 else F.FLUX_EULER_ROE_EF_DENSITY
        rng = np.random.default_rng(i)
        left = (rng.uniform(0.8, 1.2), 0.0, rng.uniform(0.8, 1.2))
        right = (0.125 * rng.uniform(0.8, 1.2), 0.0, 0.1 * rng.uniform(0.8, 1.2))
        reqs.append(case(n, kind, left, right))
    srv = F.fqnm_server_create(64 << 20, 32)
    outs = []
    try:
        for r, prob, op, st0 in reqs:
            out = np.empty((3, prob.n), np.int64)
            outs.append(out)
            F.fqnm_server_submit(srv, prob, F.density_only_raw(*st0), r.steps, out)
        F.fqnm_server_drain(srv, 300.0)
        comps = F.fqnm_server_poll(srv, 64)
    finally:
        F.fqnm_server_destroy(srv)
    assert len(comps) == len(reqs) and all(c["status"] == 0 for c in comps)
    for (r, prob, op, st0), out in zip(reqs, outs):
        ref = O.step_euler_density(op, *st0, r.steps)
        got = F.density_only_state(out)
        assert np.array_equal(got[0], ref[0]), prob.n
        assert same_bits(got[1], ref[1]) and same_bits(got[2], ref[2]), prob.n
