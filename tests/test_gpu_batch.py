"""GPU parity of batched execution: every instance of a mixed batch must end
bit-identical to the oracle run of that instance alone (and to the
per-instance comparison loop).  Sizes cover the register-resident envelope,
its edges, short-lane layouts and instances routed to the single-grid path."""
import numpy as np
import pytest

import oracle as O
from paper_2604_06947_amd import fqnm as F
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.gpu

KIND_F2O = {F.FLUX_UPWIND: O.UPWIND, F.FLUX_BURGERS_EO: O.BURGERS_EO,
            F.FLUX_BURGERS_GODUNOV: O.BURGERS_GODUNOV, F.FLUX_LF_BURGERS: O.LF_BURGERS,
            F.FLUX_BURGERS_MURMAN_ROE: O.BURGERS_MURMAN_ROE}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    F.lib()


def instance(k, n, steps, flux, bc, seed, lut=False):
    u0 = W.random_smooth_step(n, seed=seed, b=0.2)
    delta = 1e-4
    umax = float(np.max(np.abs(u0)))
    a, alpha = 1.0, 0.0
    if flux == F.FLUX_UPWIND:
        a = 1.0 if k % 2 == 0 else -0.7
        lam = 0.5 if a > 0 else 0.9 / 0.7
    elif flux == F.FLUX_LF_BURGERS:
        alpha = 1.25 * umax
        lam = 0.8 / alpha
    else:
        lam = 0.45 / umax
    prob = F.make_problem(flux, delta, lam, n, bc=bc, itype=F.I32,
                          eval_=F.EVAL_LUT if lut else F.EVAL_DIRECT, a=a, alpha=alpha)
    q0 = O.quantise(u0, delta, 32)
    op = O.Problem(KIND_F2O[flux], delta, lam, bc=bc, width=32, a=a, alpha=alpha)
    return prob, q0, steps, op


def mixed_batch():
    rng = np.random.default_rng(44)
    sizes = [1, 2, 3, 5, 63, 64, 65, 127, 128, 129, 511, 512, 513, 1023, 1024, 1025, 1026,
             2047, 2049, 4099, 8191, 16385, 32767, 32768, 32769, 65535, 65536, 65537, 70001]
    fluxes = [F.FLUX_UPWIND, F.FLUX_BURGERS_EO, F.FLUX_BURGERS_GODUNOV,
              F.FLUX_BURGERS_MURMAN_ROE, F.FLUX_LF_BURGERS]
    insts = []
    for k, n in enumerate(sizes):
        for f_i, flux in enumerate(fluxes):
            if n > 20000 and f_i > 1 and (k + f_i) % 3:
                continue  # keep the oracle time bounded
            steps = int(rng.integers(0, 60)) if n > 20000 else int(rng.integers(0, 400))
            bc = F.BC_PERIODIC if (k + f_i) % 2 == 0 else F.BC_OUTFLOW
            lut = flux in (F.FLUX_UPWIND, F.FLUX_BURGERS_EO) and k % 7 == 3
            insts.append(instance(len(insts), n, steps, flux, bc, seed=1000 + len(insts), lut=lut))
    return insts


def test_mixed_batch_matches_oracle_and_per_instance_loop():
    insts = mixed_batch()
    probs = [p for p, _, _, _ in insts]
    h = F.fqnm_batch_create(probs, [q.astype(np.int32) for _, q, _, _ in insts],
                            [s for _, _, s, _ in insts])
    try:
        F.fqnm_batch_run(h)
        got = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
        # run again from the initial states: identical
        F.fqnm_batch_reset(h)
        F.fqnm_batch_run(h)
        again = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
        F.fqnm_batch_reset(h)
        F.fqnm_batch_run_per_instance(h)
        solo = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
    finally:
        F.fqnm_batch_destroy(h)
    for i, (p, q0, steps, op) in enumerate(insts):
        ref = O.step(op, q0, steps)
        assert np.array_equal(got[i], ref), (i, p.n, p.flux, p.bc, steps)
        assert np.array_equal(again[i], ref), i
        assert np.array_equal(solo[i], ref), i


@pytest.mark.parametrize("sizes", [[5, 300, 1025, 4099, 16384], [20000, 30000], [40000, 65536],
                                   [16385, 32768, 40000, 65536], [100, 200, 20000, 30000]])
def test_batches_of_some_classes(sizes):
    """Resident instances run in one of three persistent kernels launched side
    by side: up to 16384 cells (512 threads); split kinds of 16385..32768 cells
    (512 threads, 64 cells per lane); larger split instances and two-point
    instances above 16384 cells (1024 threads).  Fluxes cycle upwind, EO,
    Godunov.  Batches here hold only the first class, only the second, only
    the third, the second and third with an instance routed to the
    single-grid path (40000 cells of a two-point kind), and all three."""
    fluxes = [F.FLUX_UPWIND, F.FLUX_BURGERS_EO, F.FLUX_BURGERS_GODUNOV]
    insts = [instance(k, n, 40 + 7 * k, fluxes[k % 3], F.BC_PERIODIC if k % 2 else F.BC_OUTFLOW,
                      seed=3000 + k) for k, n in enumerate(sizes)]
    probs = [p for p, _, _, _ in insts]
    h = F.fqnm_batch_create(probs, [q.astype(np.int32) for _, q, _, _ in insts],
                            [s for _, _, s, _ in insts])
    try:
        F.fqnm_batch_run(h)
        got = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
    finally:
        F.fqnm_batch_destroy(h)
    for i, (p, q0, steps, op) in enumerate(insts):
        assert np.array_equal(got[i], O.step(op, q0, steps)), (i, p.n, p.flux)


def test_w4_sample_of_the_4096_instance_batch():
    """The first 48 instances of the seeded 4096-instance workload (full step
    counts) run as one batch must each equal the oracle."""
    ws = W.w4_batch(count=48)
    probs, q0s, steps, ops = [], [], [], []
    for w in ws:
        probs.append(F.make_problem(w.kind, w.delta, w.lam, w.n, itype=F.I32, a=w.a))
        q0 = O.quantise(w.u0, w.delta, 32)
        q0s.append(q0)
        steps.append(w.steps)
        ops.append(O.Problem(O.UPWIND if w.kind == W.UPWIND else O.BURGERS_EO, w.delta, w.lam,
                             width=32, a=w.a))
    h = F.fqnm_batch_create(probs, [q.astype(np.int32) for q in q0s], steps)
    try:
        F.fqnm_batch_run(h)
        got = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
    finally:
        F.fqnm_batch_destroy(h)
    for i in range(len(ws)):
        if ws[i].n * ws[i].steps > 6e7:
            continue  # bounded oracle time; the property check below still applies
        assert np.array_equal(got[i], O.step(ops[i], q0s[i], steps[i])), i
    for i in range(len(ws)):
        assert int(got[i].sum()) == int(q0s[i].sum())


def test_w4_full_batch_as_benchmarked():
    """All 4096 instances of the seeded workload in one batch, as the
    benchmark runs them: every instance equals the same instance advanced
    alone by the single-grid stepper and conserves its sum (periodic), and a
    seeded sample of 32 instances, drawn among those with at most 10^7
    cell-updates, equals the oracle."""
    ws = W.w4_batch()
    probs = [F.make_problem(w.kind, w.delta, w.lam, w.n, itype=F.I32, a=w.a) for w in ws]
    q0s = [O.quantise(w.u0, w.delta, 32) for w in ws]
    steps = [w.steps for w in ws]
    h = F.fqnm_batch_create(probs, [q.astype(np.int32) for q in q0s], steps)
    try:
        F.fqnm_batch_run(h)
        got = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
        F.fqnm_batch_reset(h)
        F.fqnm_batch_run_per_instance(h)
        solo = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
    finally:
        F.fqnm_batch_destroy(h)
    for i in range(len(ws)):
        assert np.array_equal(got[i], solo[i]), i
        assert int(got[i].sum()) == int(q0s[i].sum()), i
    small = [i for i, w in enumerate(ws) if w.n * w.steps <= 10 ** 7]
    rng = np.random.default_rng(4096)
    for i in rng.choice(small, size=32, replace=False):
        w = ws[i]
        op = O.Problem(O.UPWIND if w.kind == W.UPWIND else O.BURGERS_EO, w.delta, w.lam,
                       width=32, a=w.a)
        assert np.array_equal(got[i], O.step(op, q0s[i], steps[i])), i


def test_batch_rejects_invalid_instances():
    p, q0, s, _ = instance(0, 100, 10, F.FLUX_UPWIND, F.BC_PERIODIC, seed=1)
    bad = F.make_problem(F.FLUX_UPWIND, 1e-4, 3.0, 100, itype=F.I32)  # CFL > 1
    with pytest.raises(F.FqnmError) as e:
        F.fqnm_batch_create([p, bad], [q0.astype(np.int32)] * 2, [s, s])
    assert e.value.status == F.ERR_CFL


@pytest.mark.parametrize("width", [32, 64])
def test_tiled_instances_run_together_and_match_oracle(width):
    """Instances outside the register-resident envelope (tabulated maps,
    64-bit states, more than 65536 cells) run as tiled work items, one launch
    per step block for all of them: every one equals the oracle and the
    per-instance loop."""
    ws = W.w4_tiled_mix(count=24, seed=9, width=width, nmin=1 << 10, nmax=1 << 17, smin=50,
                        smax=300)
    itype = F.I32 if width == 32 else F.I64
    dt = np.int32 if width == 32 else np.int64
    probs, q0s, ops = [], [], []
    for w in ws:
        probs.append(F.make_problem(w.kind, w.delta, w.lam, w.n, itype=itype, a=w.a,
                                    eval_=F.EVAL_LUT if w.extra["lut"] else F.EVAL_DIRECT))
        q0s.append(O.quantise(w.u0, w.delta, width))
        ops.append(O.Problem(O.UPWIND if w.kind == W.UPWIND else O.BURGERS_EO, w.delta, w.lam,
                             width=width, a=w.a))
    steps = [w.steps for w in ws]
    h = F.fqnm_batch_create(probs, [q.astype(dt) for q in q0s], steps)
    try:
        F.fqnm_batch_run(h)
        got = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
        F.fqnm_batch_reset(h)
        F.fqnm_batch_run(h)
        again = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
        F.fqnm_batch_reset(h)
        F.fqnm_batch_run_per_instance(h)
        solo = [F.fqnm_batch_get_state(h, i, p).astype(np.int64) for i, p in enumerate(probs)]
    finally:
        F.fqnm_batch_destroy(h)
    for i in range(len(ws)):
        ref = O.step(ops[i], q0s[i], steps[i], omp=True)
        assert np.array_equal(got[i], ref), (i, ws[i].n, ws[i].extra)
        assert np.array_equal(again[i], ref), i
        assert np.array_equal(solo[i], ref), i


def test_layouts_give_the_same_integers_and_autotune_keeps_them():
    """Every batch layout (class boundary, lanes per resident instance, wide
    split class, tiled cells per lane and depth) computes the same integers;
    the autotuner picks one of them, resets the instances and remembers it."""
    ws = W.w4_batch(count=40, seed=21, smax=600)
    ws += W.w4_tiled_mix(count=6, seed=22, nmin=1 << 10, nmax=1 << 17, smin=50, smax=200)
    probs, q0s, ops = [], [], []
    for w in ws:
        lut = w.extra.get("lut", False)
        probs.append(F.make_problem(w.kind, w.delta, w.lam, w.n, itype=F.I32, a=w.a,
                                    eval_=F.EVAL_LUT if lut else F.EVAL_DIRECT))
        q0s.append(O.quantise(w.u0, w.delta, 32))
        ops.append(O.Problem(O.UPWIND if w.kind == W.UPWIND else O.BURGERS_EO, w.delta, w.lam,
                             width=32, a=w.a))
    steps = [w.steps for w in ws]
    refs = [O.step(op, q0, s, omp=True) for op, q0, s in zip(ops, q0s, steps)]
    layouts = [dict(), dict(class0_max_cells=8192, class0_lanes=128, wide_split_class=2),
               dict(class0_lanes=256, tiled_vec=8, tiled_depth=48),
               dict(class0_max_cells=16384, class0_lanes=512, wide_split_class=1, tiled_vec=4,
                    tiled_depth=24)]
    h = F.fqnm_batch_create(probs, [q.astype(np.int32) for q in q0s], steps)
    try:
        for lay in layouts:
            F.fqnm_batch_set_config(h, **lay)
            F.fqnm_batch_reset(h)
            F.fqnm_batch_run(h)
            for i, p in enumerate(probs):
                assert np.array_equal(F.fqnm_batch_get_state(h, i, p).astype(np.int64),
                                      refs[i]), (lay, i)
        with pytest.raises(F.FqnmError):
            F.fqnm_batch_set_config(h, class0_lanes=100)
        cfg = F.fqnm_batch_autotune(h)
        for i, p in enumerate(probs):  # reset to the initial states
            assert np.array_equal(F.fqnm_batch_get_state(h, i, p).astype(np.int64), q0s[i])
        F.fqnm_batch_run(h)
        for i, p in enumerate(probs):
            assert np.array_equal(F.fqnm_batch_get_state(h, i, p).astype(np.int64), refs[i])
    finally:
        F.fqnm_batch_destroy(h)
    h2 = F.fqnm_batch_create(probs, [q.astype(np.int32) for q in q0s], steps)
    try:
        assert F.fqnm_batch_get_config(h2) == cfg  # remembered for batches of this shape
    finally:
        F.fqnm_batch_destroy(h2)


def test_direct_launches_match_the_graph(monkeypatch):
    """With FQNM_BATCH_NO_GRAPH set at create the batch issues its launches
    directly instead of replaying the captured graph: the same integers."""
    insts = [instance(k, n, 30 + k, [F.FLUX_UPWIND, F.FLUX_BURGERS_EO][k % 2], F.BC_PERIODIC,
                      seed=5000 + k, lut=(k == 3)) for k, n in enumerate([300, 5000, 20000, 70001])]
    probs = [p for p, _, _, _ in insts]
    monkeypatch.setenv("FQNM_BATCH_NO_GRAPH", "1")
    h = F.fqnm_batch_create(probs, [q.astype(np.int32) for _, q, _, _ in insts],
                            [s for _, _, s, _ in insts])
    monkeypatch.delenv("FQNM_BATCH_NO_GRAPH")
    try:
        for _ in range(2):
            F.fqnm_batch_reset(h)
            F.fqnm_batch_run(h)
            for i, (p, q0, steps, op) in enumerate(insts):
                assert np.array_equal(F.fqnm_batch_get_state(h, i, p).astype(np.int64),
                                      O.step(op, q0, steps)), i
    finally:
        F.fqnm_batch_destroy(h)
