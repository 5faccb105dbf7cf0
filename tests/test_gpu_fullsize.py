"""Full-size element-by-element parity of every benchmarked workload.

The expected final states are the oracle's, run once on the host by
tests/golden/make_digests.py and stored as SHA-256 digests (with the exact
sum of the first component) in tests/golden/full_size_digests.txt.  Each test
runs the workload through the C ABI at its full size, in the launch plan the
benchmark times, hashes the final device state (as little-endian int64) and
compares: a digest match is bit-for-bit equality of every cell.
"""
import hashlib
import os

import numpy as np
import pytest

from paper_2604_06947_amd import fqnm as F
from paper_2604_06947_amd import plans
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "full_size_digests.txt")


def digests():
    d = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, n, steps, s, h = line.split()
            d[k] = (int(n), int(steps), int(s), h)
    return d


D = digests()


def sha(q):
    return hashlib.sha256(np.ascontiguousarray(q, dtype="<i8").tobytes()).hexdigest()


def check(key, q, n, steps):
    en, es, esum, eh = D[key]
    assert (en, es) == (n, steps), key
    q = np.asarray(q, dtype=np.int64)
    first = q.reshape(-1) if q.ndim == 1 else q[0]
    assert int(first.sum()) == esum, f"{key}: sum of the first component differs"
    assert sha(q) == eh, f"{key}: state differs from the oracle"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    F.lib()


def run_single(prob, u0, steps, plan):
    h = F.fqnm_create_from_field(prob, u0)
    try:
        if plan is not None:
            F.fqnm_set_plan(h, *plan)
        F.fqnm_step(h, steps)
        return F.fqnm_get_state(h, prob)
    finally:
        F.fqnm_destroy(h)


def test_w1_full():
    w = W.w1_advection_square()
    prob = F.make_problem(F.FLUX_UPWIND, w.delta, w.lam, w.n, itype=F.I32, a=w.a)
    check("w1", run_single(prob, w.u0, w.steps, None), w.n, w.steps)


@pytest.mark.parametrize("plan", [plans.BENCH_PLAN_W2, (F.KERNEL_STREAM, 4, 1)])
def test_w2_full(plan):
    w = W.w2_burgers_step()
    print("w2 plan", plan, flush=True)
    prob = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam, w.n, itype=F.I32,
                          eval_=F.EVAL_LUT)
    check("w2", run_single(prob, w.u0, w.steps, plan), w.n, w.steps)


@pytest.mark.parametrize("r", [1e-2, 1e-3, 1e-4])
@pytest.mark.parametrize("plan", [plans.BENCH_PLAN_W3, plans.STREAM_PLAN_W3])
def test_w3_full(r, plan):
    w = W.w3_nyquist_advection(r=r)
    print("w3", r, plan, flush=True)
    prob = F.make_problem(F.FLUX_UPWIND, w.delta, w.lam, w.n, itype=F.I64, a=w.a)
    check(f"w3_r{r:g}", run_single(prob, w.u0, w.steps, plan), w.n, w.steps)


@pytest.mark.parametrize("which", ["tb", "march"])
def test_w6_full(which):
    w = W.w6_burgers_2d()
    ny, nx = w.shape
    q0 = F.fqnm_quantise(w.u0.ravel(), w.delta, F.I32).reshape(w.shape)
    axes = [F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam[m], (nx, ny)[m], itype=F.I32)
            for m in range(2)]
    h = F.fqnm_create_nd(axes, q0)
    try:
        if which == "tb":
            kern, vec, K, rows = plans.ND_PLAN_W6
            F.fqnm_set_plan(h, kern, vec, F.nd_tb_depth(K, rows))
        else:
            vec, rows = plans.ND_MARCH_PLAN_W6
            F.fqnm_set_plan(h, F.KERNEL_ND_MARCH, vec, rows)
        F.fqnm_step(h, w.steps)
        p = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam[0], nx * ny, itype=F.I32)
        q = F.fqnm_get_state(h, p)
    finally:
        F.fqnm_destroy(h)
    check("w6", q.reshape(-1), nx * ny, w.steps)


def test_w4_full_batch():
    ws = W.w4_batch()
    sizes = [w.n for w in ws]
    q_all = F.fqnm_quantise(np.concatenate([w.u0 for w in ws]), ws[0].delta, F.I32)
    q0s = np.split(q_all, np.cumsum(sizes)[:-1])
    probs = [F.make_problem(w.kind, w.delta, w.lam, w.n, itype=F.I32, a=w.a) for w in ws]
    h = F.fqnm_batch_create(probs, q0s, [w.steps for w in ws])
    try:
        F.fqnm_batch_run(h)
        bad = []
        for k, (w, p) in enumerate(zip(ws, probs)):
            q = F.fqnm_batch_get_state(h, k, p)
            en, es, esum, eh = D[f"w4_{k}"]
            if (en, es) != (w.n, w.steps) or sha(q) != eh:
                bad.append(k)
    finally:
        F.fqnm_batch_destroy(h)
    assert not bad, f"{len(bad)} instances differ from the oracle, first {bad[:8]}"


def test_w5_full_served_mix():
    """The served Sod requests that have oracle digests (every request of at
    most 16384 cells, the largest request and seven more of the larger ones),
    submitted together to one server with the benchmark's 64 MiB budget: each
    result, computed in the mix, equals the oracle's run of that request alone."""
    reqs = W.w5_sod_requests()
    keys = sorted((int(k[3:]) for k in D if k.startswith("w5_")))
    assert len(keys) >= 500 and max(r.n for r in reqs) in [reqs[i].n for i in keys]
    srv = F.fqnm_server_create(64 << 20, 64)
    outs = {}
    try:
        for i in keys:
            r = reqs[i]
            q0 = F.fqnm_quantise(r.U0.ravel(), r.delta, F.I64)
            prob = F.make_problem(r.kind, r.delta, r.lam, r.n, bc=F.BC_OUTFLOW, itype=F.I64,
                                  gamma=r.gamma)
            outs[i] = np.empty_like(q0)
            F.fqnm_server_submit(srv, prob, q0, r.steps, outs[i])
        F.fqnm_server_drain(srv, 110.0)
        comps = []
        while True:
            c = F.fqnm_server_poll(srv, 256)
            if not c:
                break
            comps += c
    finally:
        F.fqnm_server_destroy(srv)
    assert len(comps) == len(keys) and all(c["status"] == 0 for c in comps)
    bad = []
    for i in keys:
        r = reqs[i]
        q = outs[i].reshape(3, r.n)
        en, es, esum, eh = D[f"w5_{i}"]
        if (en, es) != (r.n, r.steps) or sha(q) != eh or int(q[0].sum()) != esum:
            bad.append(i)
    assert not bad, f"{len(bad)} served requests differ from the oracle, first {bad[:8]}"
