"""Benchmark of the FQNM integer-transfer hot path on one MI355X.

Headline workload (one "step" of this benchmark = one complete solve):
  inviscid Burgers, 2^20 int32 cells, delta = 1e-5, CFL 0.45, Engquist-Osher
  transfer tabulated over the visited range, 10000 time steps, periodic;
  the initial state is resident in HBM (restored by a device copy inside the
  timed region) and the table is built once at create.
Metric: cell-updates/s (cells x time steps per second).

Also reported on the same line: the roofline of the dominant kernel, the CPU
oracle (single thread and all host cores) on bounded samples, and the other
workloads: the first workload's latency, near-Nyquist int64 advection with
the one-step streaming kernel and with temporal blocking, the FP64 twin, the
4096-instance batch, 1000 served Sod requests, 2-D Burgers, single-grid Sod
and level statistics.  Final states of the benchmarked runs are checked
against the oracle's full-size digests (tests/golden/full_size_digests.txt,
written from the oracle by tests/golden/make_digests.py; reading that file
runs nothing of the oracle).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
       python bench.py --copy-probe   (a plain device copy of known size, for
                                       scaling rocprofv3 byte counters)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector ALU issue peak of MI355X: 256 CUs x 4 SIMDs, a wave64 instruction
# every 4 cycles per SIMD (16 lanes), 2.4 GHz -> 64 lane-operations per CU and
# cycle: 3.93e13 integer (or non-FMA FP64) operations per second.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
SIMDS, CLOCK_HZ = 1024, 2.4e9
FP64_PEAK_TFLOPS = 78.6
# Operations per cell-update of the split update as Sec. 2.4 counts them: two
# map evaluations and one addition per interface, two subtractions per cell
# (a tabulated map evaluation is one table read).
OPS_PER_CELL_UPDATE = 5
GOLDEN = os.path.join(ROOT, "tests", "golden", "full_size_digests.txt")


def golden():
    """Expected final-state digests written from the oracle (key -> (n, steps, sum, sha))."""
    d = {}
    if os.path.exists(GOLDEN):
        for line in open(GOLDEN):
            if line.strip() and not line.startswith("#"):
                k, n, st, sm, h = line.split()
                d[k] = (int(n), int(st), int(sm), h)
    return d


def state_sha(q):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(q, dtype="<i8").tobytes()).hexdigest()


def parity(key, q, G):
    """True/False against the stored oracle digest, None when there is none."""
    if key not in G:
        return None
    return state_sha(q) == G[key][3]


def counter_fields(plans, key, launch_s):
    """Counter-derived figures of a timed kernel: HBM bytes per launch and their
    share of the 8 TB/s peak over the measured launch time, VALU issue (one
    wave64 instruction per SIMD every 4 cycles) and LDS bank-conflict share.
    null when the counters were taken on other kernel sources."""
    c = plans.COUNTERS[key]
    valid = c["sources_sha"] is not None and kernel_sources_sha(c["sources"]) == c["sources_sha"]
    tb = c["traffic_bytes"] if valid else None
    vi = c["valu_insts"] if valid else None
    return {"traffic": tb,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "hbm_counter_frac": tb / launch_s / (HBM_PEAK_GBS * 1e9) if tb else None,
            "valu_issue_frac": vi * 4.0 / (SIMDS * CLOCK_HZ * launch_s) if vi else None,
            "lds_bank_conflict_frac": c["lds_bank_conflict_frac"] if valid else None,
            "counters_sources_sha": c["sources_sha"]}


def kernel_sources_sha(sources=None):
    import hashlib
    from paper_2604_06947_amd import plans
    pkg = os.path.join(ROOT, "paper_2604_06947_amd")
    h = hashlib.sha256()
    for rel in sources or plans.KERNEL_SOURCES:
        with open(os.path.join(pkg, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--only", default="", help="run only this part: w2, w3, batch, batch_only "
                    "(the batched W4 run alone), serve, serve_closed (the served requests "
                    "once, closed loop), levels, nd, euler, euler_cw (componentwise Sod only)")
    return ap.parse_args()


class Solver:
    """One resident problem whose state lives in a torch tensor (borrowed by the
    library); q0 is quantised on the device once and restored per solve by a
    device copy on the stream."""

    def __init__(self, F, prob, u0, plan, stream):
        import torch
        self.F, self.prob = F, prob
        tmp = F.fqnm_create_from_field(prob, u0, stream)
        q0 = F.fqnm_get_state(tmp, prob)
        F.fqnm_destroy(tmp)
        self.q0_sum = int(q0.astype(np.int64).sum())
        self.q0 = torch.from_numpy(q0).to("cuda")
        self.cur = self.q0.clone()
        self.h = F.fqnm_create_on_device(prob, self.cur.data_ptr(), stream)
        if plan is not None:
            F.fqnm_set_plan(self.h, *plan)

    def restore(self):
        self.cur.copy_(self.q0, non_blocking=True)

    def launches(self, steps):
        p = self.F.fqnm_get_plan(self.h)
        return steps if p["kernel"] == self.F.KERNEL_STREAM else -(-steps // p["depth"])

    def close(self):
        self.F.fqnm_destroy(self.h)


def time_solver(S, steps_per_solve, K, W):
    """Returns (seconds per solve, seconds of stepping per solve from events)."""
    import torch
    F = S.F
    ev = []
    for i in range(W + K):
        if i == W:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        S.restore()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        F.fqnm_step(S.h, steps_per_solve)
        e1.record()
        if i >= W:
            ev.append((e0, e1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = sum(a.elapsed_time(b) for a, b in ev) / 1e3 / K
    return (t1 - t0) / K, step_s


def bench_twin(F, W, plans, stream, int_value, reps=3):
    """The classical split finite-volume scheme on the same Burgers workload
    with an FP64 state (Sec. 2.1), same kernels' tiling, timed like the
    headline (stepping only; the state is uploaded before the timer)."""
    import torch
    w = W.w2_burgers_step()
    prob = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam, w.n)
    ts = []
    for _ in range(reps + 1):
        h = F.fqnm_create_classical(prob, w.u0, stream)
        F.fqnm_set_plan(h, *plans.TWIN_PLAN_W2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.fqnm_step(h, w.steps)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        F.fqnm_destroy(h)
    t = float(np.median(ts[1:]))
    rate = w.n * w.steps / t
    log(f"[bench] W2 FP64 twin {rate:.3e} cell-updates/s")
    return {"w2_fp64_twin": {"cell_updates_per_s": rate, "ms_per_solve": t * 1e3,
                             "plan": list(plans.TWIN_PLAN_W2),
                             "integer_table_over_fp64": int_value / rate}}


def bench_batch(F, W, stream, G, reps=5):
    """4096 instances (advection/Burgers, 256..65536 cells, 500..5000 steps) in
    one batched run against the one-instance-at-a-time loop on the same GPU;
    every instance's final state is checked against the oracle's digest."""
    import torch
    log("[bench] W4 generating 4096 instances")
    ws = W.w4_batch()
    sizes = [w.n for w in ws]
    q_all = F.fqnm_quantise(np.concatenate([w.u0 for w in ws]), ws[0].delta, F.I32, stream)
    q0s = np.split(q_all, np.cumsum(sizes)[:-1])
    probs = [F.make_problem(w.kind, w.delta, w.lam, w.n, itype=F.I32, a=w.a) for w in ws]
    steps = [w.steps for w in ws]
    work = float(sum(n * s for n, s in zip(sizes, steps)))
    h = F.fqnm_batch_create(probs, q0s, steps, stream)
    try:
        def timed():
            F.fqnm_batch_reset(h)
            F.fqnm_batch_run(h)  # warm-up
            torch.cuda.synchronize()
            out = []
            for _ in range(reps):
                F.fqnm_batch_reset(h)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F.fqnm_batch_run(h)
                torch.cuda.synchronize()
                out.append(time.perf_counter() - t0)
            return out
        F.fqnm_batch_set_config(h)  # the default layout
        t_default = float(np.median(timed()))
        t0 = time.perf_counter()
        cfg = F.fqnm_batch_autotune(h)
        t_tune = time.perf_counter() - t0
        ts = timed()
        log(f"[bench] W4 batched {min(ts)*1e3:.1f} ms (default layout {t_default*1e3:.1f} ms, "
            f"autotuned {cfg}); per-instance loop follows")
        checked = ok = 0
        for k, p in enumerate(probs):
            r = parity(f"w4_{k}", F.fqnm_batch_get_state(h, k, p), G)
            if r is not None:
                checked += 1
                ok += bool(r)
        F.fqnm_batch_reset(h)
        F.fqnm_batch_run_per_instance(h)  # creates the per-instance contexts, warm-up
        torch.cuda.synchronize()
        F.fqnm_batch_reset(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.fqnm_batch_run_per_instance(h)
        torch.cuda.synchronize()
        t_solo = time.perf_counter() - t0
    finally:
        F.fqnm_batch_destroy(h)
    t_b = float(np.median(ts))
    return {"w4_batch": {"instances": len(ws), "cell_updates": work,
                         "batched_ms": t_b * 1e3, "batched_cell_updates_per_s": work / t_b,
                         "per_instance_ms": t_solo * 1e3,
                         "per_instance_cell_updates_per_s": work / t_solo,
                         "speedup_vs_per_instance": t_solo / t_b,
                         "layout": {"autotuned": cfg, "autotune_s": t_tune,
                                    "default_layout_ms": t_default * 1e3},
                         "parity_vs_oracle": {"checked": checked, "bit_exact": ok}}}


def bench_batch_only(F, W, stream, reps=2):
    """The batched W4 run alone, in the default layout (a short command for
    profilers: no autotuning and no per-instance loop)."""
    import torch
    ws = W.w4_batch()
    sizes = [w.n for w in ws]
    q_all = F.fqnm_quantise(np.concatenate([w.u0 for w in ws]), ws[0].delta, F.I32, stream)
    q0s = np.split(q_all, np.cumsum(sizes)[:-1])
    probs = [F.make_problem(w.kind, w.delta, w.lam, w.n, itype=F.I32, a=w.a) for w in ws]
    h = F.fqnm_batch_create(probs, q0s, [w.steps for w in ws], stream)
    try:
        ts = []
        for _ in range(reps):
            F.fqnm_batch_reset(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F.fqnm_batch_run(h)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
    finally:
        F.fqnm_batch_destroy(h)
    return {"w4_batched_only": {"batched_ms": float(np.median(ts)) * 1e3}}


def bench_tiled_mix(F, W, stream, reps=3):
    """Batches of instances outside the register-resident envelope (sizes up
    to 2^20 cells, a third tabulated; int32, and int64), which run as tiled
    work items, one launch per step block for all of them, against the
    one-instance-at-a-time loop on the same GPU."""
    import torch
    res = {}
    for width, count in ((32, 96), (64, 48)):
        ws = W.w4_tiled_mix(count=count, seed=44 + width, width=width)
        itype = F.I32 if width == 32 else F.I64
        q0s = [F.fqnm_quantise(w.u0, w.delta, itype, stream) for w in ws]
        probs = [F.make_problem(w.kind, w.delta, w.lam, w.n, itype=itype, a=w.a,
                                eval_=F.EVAL_LUT if w.extra["lut"] else F.EVAL_DIRECT) for w in ws]
        work = float(sum(w.n * w.steps for w in ws))
        h = F.fqnm_batch_create(probs, q0s, [w.steps for w in ws], stream)
        try:
            cfg = F.fqnm_batch_autotune(h)
            ts = []
            for r in range(reps + 1):
                F.fqnm_batch_reset(h)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F.fqnm_batch_run(h)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            F.fqnm_batch_reset(h)
            F.fqnm_batch_run_per_instance(h)  # creates the contexts, warm-up
            F.fqnm_batch_reset(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F.fqnm_batch_run_per_instance(h)
            torch.cuda.synchronize()
            t_solo = time.perf_counter() - t0
        finally:
            F.fqnm_batch_destroy(h)
        t_b = float(np.median(ts[1:]))
        res[f"int{width}"] = {
            "instances": count, "sizes": "log-uniform 2^12..2^20", "steps": "500..2000",
            "tabulated": sum(1 for w in ws if w.extra["lut"]), "cell_updates": work,
            "batched_ms": t_b * 1e3, "batched_cell_updates_per_s": work / t_b,
            "per_instance_cell_updates_per_s": work / t_solo,
            "speedup_vs_per_instance": t_solo / t_b, "layout": cfg}
        log(f"[bench] tiled mix int{width}: batched {work / t_b:.3e}, "
            f"per instance {work / t_solo:.3e} cell-updates/s")
    return {"w4_tiled_mix": res}


SERVE_COUNT = int(os.environ.get("FQNM_SERVE_COUNT", "1000"))
SERVE_NMAX = int(os.environ.get("FQNM_SERVE_NMAX", str(1 << 18)))
SERVE_SUBSET = int(os.environ.get("FQNM_SERVE_SUBSET", "150"))  # loads 0.5 and 0.9
FIFO_SUBSET = int(os.environ.get("FQNM_FIFO_SUBSET", "16"))     # the FIFO comparison
SERVE_BUDGET = 64 << 20


def _serve_inputs(F, W, stream):
    reqs = W.w5_sod_requests(count=SERVE_COUNT, nmax=SERVE_NMAX)
    out = []
    for r in reqs:
        q0 = F.fqnm_quantise(r.U0.ravel(), r.delta, F.I64, stream)
        prob = F.make_problem(r.kind, r.delta, r.lam, r.n, bc=F.BC_OUTFLOW, itype=F.I64,
                              gamma=r.gamma)
        out.append((prob, q0, r.steps))
    return out


def _serve_run(F, items, arrivals, tick=64):
    """Submit at the given arrival offsets (None = all at once); returns
    (wall seconds, latencies in submission order, stats, final states)."""
    srv = F.fqnm_server_create(SERVE_BUDGET, tick)
    outs = [np.empty_like(q0) for _, q0, _ in items]
    ids = []
    t0 = F.fqnm_server_now()
    try:
        for k, ((prob, q0, steps), out) in enumerate(zip(items, outs)):
            if arrivals is not None:
                wait = t0 + arrivals[k] - F.fqnm_server_now()
                if wait > 0:
                    time.sleep(wait)
            ids.append(F.fqnm_server_submit(srv, prob, q0, steps, out))
        F.fqnm_server_drain(srv, 900.0)
        t1 = F.fqnm_server_now()
        comps = []
        while True:
            c = F.fqnm_server_poll(srv, 256)
            if not c:
                break
            comps += c
        stats = F.fqnm_server_stats_get(srv)
    finally:
        F.fqnm_server_destroy(srv)
    assert all(c["status"] == 0 for c in comps)
    by_id = {c["id"]: c for c in comps}
    lat = np.array([by_id[i]["t_done"] - by_id[i]["t_submit"] for i in ids])
    stats["service_s"] = np.array([by_id[i]["t_done"] - by_id[i]["t_admit"] for i in ids])
    return t1 - t0, lat, stats, outs


def _pct(lat, svc=None):
    """p50/p99 of submit-to-done latency (queueing included) and, when given,
    of admit-to-done service time."""
    out = {"p50_latency_s": float(np.percentile(lat, 50)),
           "p99_latency_s": float(np.percentile(lat, 99))}
    if svc is not None:
        out["p50_service_s"] = float(np.percentile(svc, 50))
        out["p99_service_s"] = float(np.percentile(svc, 99))
    return out


def served_fp64_fields(cap):
    """FP64 use of the served Euler kernel (k_euler_multi) at the closed-loop
    capacity: its counters give VALU and FP64 wavefront-instructions and FP64
    FLOPs (an FMA counts two) per cell-update; times the capacity, against the
    issue rate (one wave64 instruction per SIMD every 4 cycles) and the
    78.6 TFLOP/s FP64 vector peak.  The fractions are over the whole closed
    loop, host-side tick gaps included.  null when taken on other sources."""
    from paper_2604_06947_amd import plans
    c = plans.COUNTERS["euler_multi"]
    ok = c["sources_sha"] is not None and kernel_sources_sha(c["sources"]) == c["sources_sha"]
    if not ok:
        return {"valu_issue_frac": None, "fp64_issue_frac": None, "fp64_flops_frac": None,
                "counters_sources_sha": c["sources_sha"]}
    issue = SIMDS * CLOCK_HZ / 4.0
    return {"kernel": "k_euler_multi",
            "valu_insts_per_cell_update": c["valu_insts_per_cell_update"],
            "fp64_insts_per_cell_update": c["f64_insts_per_cell_update"],
            "valu_issue_frac": c["valu_insts_per_cell_update"] * cap / issue,
            "fp64_issue_frac": c["f64_insts_per_cell_update"] * cap / issue,
            "fp64_flops_frac": c["f64_flops_per_cell_update"] * 64 * cap
            / (FP64_PEAK_TFLOPS * 1e12),
            "counters_sources_sha": c["sources_sha"]}


def bench_serve_closed(F, W, stream):
    """The served requests once, all submitted at once (closed loop): the
    profiling form of the served workload, whose cell-update total divides
    the kernel's counter totals."""
    items = _serve_inputs(F, W, stream)
    work = float(sum(p.n * s for p, _, s in items))
    t, _, st, _ = _serve_run(F, items, None)
    return {"w5_serve_closed": {"requests": len(items), "cell_updates": work,
                                "closed_loop_s": t, "cell_updates_per_s": work / t,
                                "ticks": st["ticks"]}}


def bench_serve(F, W, stream, G):
    """Config 5 as specified: SERVE_COUNT Sod requests, sizes log-uniform in
    [2^10, SERVE_NMAX], 64 MiB device budget.  Closed loop (everything
    submitted at once) gives the capacity C; Poisson arrivals at 0.7 C run on
    all requests; 0.5 C and 0.9 C, and the FIFO comparison, run on seeded
    subsets named in the result.  Served final states are checked against the
    oracle digests (every request of at most 16384 cells and 8 larger ones)."""
    import torch
    log(f"[bench] W5 {SERVE_COUNT} Sod requests, sizes 2^10..{SERVE_NMAX}")
    items = _serve_inputs(F, W, stream)
    work_of = np.array([float(p.n * s) for p, _, s in items])
    work = float(work_of.sum())
    big = int(np.argmax([p.n for p, _, _ in items]))
    t_cl, lat_cl, st_cl, outs = _serve_run(F, items, None)
    cap = work / t_cl
    checked = ok = 0
    for i, (p, _, _) in enumerate(items):
        r = parity(f"w5_{i}", outs[i], G) if SERVE_COUNT == 1000 and SERVE_NMAX == 1 << 18 else None
        if r is not None:
            checked += 1
            ok += bool(r)
    del outs
    log(f"[bench] W5 closed-loop capacity {cap:.3e} cell-updates/s ({t_cl:.1f} s); "
        f"parity {ok}/{checked}")
    res = {"requests": len(items), "sizes": f"log-uniform 2^10..{SERVE_NMAX}",
           "fp64_valu": served_fp64_fields(cap),
           "budget_bytes": SERVE_BUDGET, "cell_updates": work,
           "largest_request": {"cells": int(items[big][0].n), "steps": int(items[big][2])},
           "closed_loop_cell_updates_per_s": cap, "closed_loop_s": t_cl,
           "closed_loop_p50_s": float(np.percentile(lat_cl, 50)),
           "closed_loop_p99_s": float(np.percentile(lat_cl, 99)),
           "peak_bytes": st_cl["peak_bytes"], "ticks": st_cl["ticks"],
           "parity_vs_oracle": {"checked": checked, "bit_exact": ok}}
    rate = 0.7 * cap / (work / len(items))
    arr = W.poisson_arrivals(len(items), rate, seed=55)
    t, lat, st7, _ = _serve_run(F, items, arr)
    res["load0.7"] = {"requests": "all", "arrival_rate_per_s": rate,
                      "cell_updates_per_s": work / t, **_pct(lat, st7["service_s"])}
    log(f"[bench] W5 load 0.7: p50 {np.percentile(lat, 50):.3f}s p99 {np.percentile(lat, 99):.3f}s")
    rng = np.random.default_rng(77)
    sub = sorted(int(i) for i in rng.choice(len(items), size=min(SERVE_SUBSET, len(items)),
                                            replace=False))
    sub_items = [items[i] for i in sub]
    sub_work = float(work_of[sub].sum())
    for load in (0.5, 0.9):
        rate = load * cap / (sub_work / len(sub))
        arr = W.poisson_arrivals(len(sub), rate, seed=55)
        t, lat, stl, _ = _serve_run(F, sub_items, arr)
        res[f"load{load}"] = {
            "requests": f"{len(sub)} drawn with numpy default_rng(77).choice "
                        f"({len(items)}, {len(sub)}, replace=False)",
            "arrival_rate_per_s": rate, "cell_updates_per_s": sub_work / t,
            **_pct(lat, stl["service_s"])}
        log(f"[bench] W5 load {load} (subset): p50 {np.percentile(lat, 50):.3f}s "
            f"p99 {np.percentile(lat, 99):.3f}s")
    # FIFO: one request at a time through the single-grid stepper, against the
    # served closed loop on the same seeded subset: drawn from all requests,
    # and drawn from those of at most 2^14 cells (which cannot fill the GPU
    # alone: the regime batching is for)
    small = [i for i, (p, _, _) in enumerate(items) if p.n <= 1 << 14]
    for key, pool, seed, size in (("fifo", list(range(len(items))), 78, FIFO_SUBSET),
                                  ("fifo_small", small, 79, 4 * FIFO_SUBSET)):
        rng = np.random.default_rng(seed)
        size = min(size, len(pool))
        fsub = sorted(int(pool[i]) for i in rng.choice(len(pool), size=size, replace=False))
        f_items = [items[i] for i in fsub]
        f_work = float(work_of[fsub].sum())
        t_srv, _, _, _ = _serve_run(F, f_items, None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for prob, q0, steps in f_items:
            h = F.fqnm_create(prob, q0, stream)
            F.fqnm_step(h, steps)
            F.fqnm_get_state(h, prob)
            F.fqnm_destroy(h)
        t_fifo = time.perf_counter() - t0
        what = "all requests" if key == "fifo" else "the requests of at most 2^14 cells"
        res[key] = {"requests": f"{size} of {what} ({len(pool)}), drawn with numpy "
                                f"default_rng({seed}).choice({len(pool)}, {size}, replace=False)",
                    "fifo_one_at_a_time_cell_updates_per_s": f_work / t_fifo,
                    "served_closed_loop_cell_updates_per_s": f_work / t_srv,
                    "served_vs_fifo": t_fifo / t_srv}
        log(f"[bench] W5 {key}: FIFO {f_work / t_fifo:.3e} against served "
            f"{f_work / t_srv:.3e} cell-updates/s")
    return {"w5_serve": res}


def bench_nd(F, W, plans, stream, G, reps=3):
    """W6: 2-D Burgers by directional composition, 4096 x 4096 int32 cells,
    1000 steps; the marching kernel with temporal blocking (several steps per
    launch), and the one-step-per-launch marching kernel beside it.  Device
    time of the whole solve by HIP events on the library's stream (the state
    is uploaded before the timer)."""
    import torch
    w = W.w6_burgers_2d()
    ny, nx = w.shape
    cells = nx * ny
    q0 = F.fqnm_quantise(w.u0.ravel(), w.delta, F.I32, stream).reshape(w.shape)
    axes = [F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam[m], (nx, ny)[m], itype=F.I32)
            for m in range(2)]

    flat = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam[0], cells, itype=F.I32)
    par = {}

    def solve(kernel, vec, depth):
        ts, inv = [], None
        for rep in range(reps + 1):
            h = F.fqnm_create_nd(axes, q0, stream)
            F.fqnm_set_plan(h, kernel, vec, depth)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(torch.cuda.current_stream())
            F.fqnm_step(h, w.steps)
            e1.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
            inv = F.fqnm_invariants_get(h)
            if rep == reps:
                par[kernel] = parity("w6", F.fqnm_get_state(h, flat), G)
            F.fqnm_destroy(h)
        return float(np.median(ts[1:])), inv

    kern, vec, K, rows = plans.ND_PLAN_W6
    assert w.steps % K == 0
    t, inv = solve(kern, vec, F.nd_tb_depth(K, rows))
    launches = w.steps // K
    rate = cells * w.steps / t
    ach = 8.0 * cells * K / (t / launches) / 1e9
    mv, mr = plans.ND_MARCH_PLAN_W6
    t1, inv1 = solve(F.KERNEL_ND_MARCH, mv, mr)
    log(f"[bench] W6 2-D {rate:.3e} cell-updates/s ({K} steps per launch), {ach:.0f} GB/s "
        f"algorithmic; one step per launch {cells * w.steps / t1:.3e}")
    cb = counter_fields(plans, "w6", t / launches)
    return {"w6_burgers_2d": {
        "cells": cells, "shape": [ny, nx], "time_steps": w.steps, "cell_updates_per_s": rate,
        "ms_per_solve": t * 1e3, "plan": {"vec": vec, "steps_per_launch": K, "rows": rows},
        "kernel": "k_nd_tb<int, P_EO, %d, %d, true, false>" % (vec, K),
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "bytes_per_cell_update": 8,
                     "algorithmic_bytes_per_launch": 8 * cells * K,
                     "avg_launch_us": t / launches * 1e6, **cb},
        "parity_vs_oracle": {"temporally_blocked": par.get(kern),
                             "one_step_per_launch": par.get(F.KERNEL_ND_MARCH)},
        "one_step_per_launch": {"kernel": "k_nd_march<int, P_EO, %d, 2>" % mv, "rows": mr,
                                "cell_updates_per_s": cells * w.steps / t1,
                                "avg_launch_us": t1 / w.steps * 1e6},
        "conservation_ok": inv["sum"][0] == int(q0.astype(np.int64).sum())
        and inv1["sum"][0] == inv["sum"][0]}}


def euler_counter_fields(plans, launch_s):
    """FP64 figures of k_euler_step (componentwise Sod, 2^20 cells, 8 steps
    per launch) from its counters: VALU issue, the FP64 share of the VALU
    instructions, FP64 issue and FP64 FLOP/s against the 78.6 TFLOP/s vector
    peak (an FMA counts two).  null when taken on other kernel sources."""
    c = plans.COUNTERS["euler_step"]
    ok = c["sources_sha"] is not None and kernel_sources_sha(c["sources"]) == c["sources_sha"]
    if not ok:
        return {"valu_issue_frac": None, "fp64_share_of_valu": None, "fp64_issue_frac": None,
                "fp64_flops_frac": None, "counters_sources_sha": c["sources_sha"]}
    slots = SIMDS * CLOCK_HZ * launch_s / 4.0
    return {"valu_issue_frac": c["valu_insts"] / slots,
            "fp64_share_of_valu": c["f64_insts"] / c["valu_insts"],
            "fp64_issue_frac": c["f64_insts"] / slots,
            "fp64_flops_frac": c["f64_flops"] * 64 / launch_s / (FP64_PEAK_TFLOPS * 1e12),
            "counters_sources_sha": c["sources_sha"]}


def bench_euler(F, W, stream, n=1 << 20, steps=200, reps=3, kinds=("componentwise",
                                                                     "density_only")):
    """Sod at 2^20 cells, 200 steps of the single-grid Euler kernel: the
    componentwise quantisation (all of rho, m, E counted) and the density-only
    prototype (FP64 m and E).  Device time of the steps by HIP events."""
    import torch
    from paper_2604_06947_amd import plans
    out = {}
    for tag, kind in (("componentwise", F.FLUX_EULER_ROE_EF),
                      ("density_only", F.FLUX_EULER_ROE_EF_DENSITY)):
        if tag not in kinds:
            continue
        r = W.sod_request(n, kind=6)
        prob = F.make_problem(kind, r.delta, r.lam, n, bc=F.BC_OUTFLOW, itype=F.I64, gamma=1.4)
        ts = []
        for _ in range(reps + 1):
            h = F.fqnm_create_from_field(prob, r.U0.ravel(), stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(torch.cuda.current_stream())
            F.fqnm_step(h, steps)
            e1.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
            F.fqnm_destroy(h)
        t = float(np.median(ts[1:]))
        rate = n * steps / t
        ach = 48.0 * n / (t / steps) / 1e9
        log(f"[bench] Sod {tag} {rate:.3e} cell-updates/s")
        out[f"sod_2e20_{tag}"] = {"cell_updates_per_s": rate, "ms_per_step": t / steps * 1e3,
                                  "kernel_GBps_algorithmic": ach,
                                  "frac_of_hbm": ach / HBM_PEAK_GBS,
                                  "bound": "fp64 alu (divisions, square roots)"}
        if tag == "componentwise":
            out[f"sod_2e20_{tag}"]["counters"] = euler_counter_fields(plans, t / steps * 8)
    return out


def bench_levels(F, W, stream, reps=5):
    """Level statistics at the headline size (2^20 int32 cells, Burgers EO after
    2000 steps): histogram + entropy, and one transition step with its counts
    and row-sum defect.  Wall clock per call (device sort, host sums, copies
    and the per-call temporary allocations included).  Returns the extras and
    the state the statistics were taken on (the CPU leg times the oracle on it)."""
    w = W.w2_burgers_step()
    prob = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam, w.n, itype=F.I32, eval_=F.EVAL_LUT)
    h = F.fqnm_create_from_field(prob, w.u0, stream)
    try:
        F.fqnm_step(h, 2000)
        q = F.fqnm_get_state(h, prob).astype(np.int64)
        F.fqnm_entropy(h)
        t0 = time.perf_counter()
        for _ in range(reps):
            S, _ = F.fqnm_entropy(h)
        t_ent = (time.perf_counter() - t0) / reps
        nl = F.fqnm_level_histogram(h)[0].size
        F.fqnm_step_transitions(h, w.n)
        t0 = time.perf_counter()
        for _ in range(reps):
            _, _, c, rho = F.fqnm_step_transitions(h, w.n)
        t_tr = (time.perf_counter() - t0) / reps
    finally:
        F.fqnm_destroy(h)
    return {"levels_w2": {
        "cells": w.n, "occupied_levels": int(nl), "entropy": S, "transition_pairs": int(c.size),
        "row_defect": rho,
        "entropy_ms": t_ent * 1e3, "entropy_cells_per_s": w.n / t_ent,
        "transitions_ms": t_tr * 1e3, "transitions_cells_per_s": w.n / t_tr}}, q


def cpu_baseline(W, level_state=None):
    """The CPU leg: the oracle as it stands, timed on this host's cores on
    bounded samples of the benchmarked workloads -- the plain single-threaded
    build and the OpenMP build of the same source on all available cores."""
    import oracle as O
    model, avail = host_cpu()
    omp_threads = O.threads(omp=True)
    res = {}

    def scalar_rate(w, steps, omp):
        op = O.Problem(w.kind, w.delta, w.lam, bc=w.bc, width=w.width, a=w.a)
        q0 = O.quantise(w.u0, w.delta, w.width)
        t0 = time.perf_counter()
        O.step(op, q0, steps, omp=omp)
        dt = time.perf_counter() - t0
        return w.n * steps / dt, dt

    w2 = W.w2_burgers_step()
    s1 = int(os.environ.get("FQNM_CPU_SAMPLE_STEPS", "1500"))
    log(f"[bench] cpu oracle: W2 {w2.n} cells x {s1} steps, one thread")
    r1, d1 = scalar_rate(w2, s1, False)
    log(f"[bench] cpu oracle: W2 {w2.n} cells x {w2.steps} steps, {omp_threads} threads")
    rA, dA = scalar_rate(w2, w2.steps, True)
    res["w2_single_thread"] = {"value": r1, "cores": 1, "seconds": d1,
                               "sample": f"2^20 cells x {s1} of the {w2.steps} steps"}
    res["w2_all_cores"] = {"value": rA, "cores": omp_threads, "seconds": dA,
                           "sample": "the whole workload, 2^20 cells x 10000 steps"}
    w3 = W.w3_nyquist_advection(r=1e-3)
    r3, d3 = scalar_rate(w3, 40, True)
    res["w3_all_cores"] = {"value": r3, "cores": omp_threads, "seconds": d3,
                           "sample": "2^24 int64 cells x 40 of the 2000 steps (delta/dx = 1e-3)"}
    ws = W.w4_batch()[:32]
    t0 = time.perf_counter()
    for w in ws:
        op = O.Problem(w.kind, w.delta, w.lam, bc=w.bc, width=w.width, a=w.a)
        O.step(op, O.quantise(w.u0, w.delta, w.width), w.steps)
    d4 = time.perf_counter() - t0
    res["w4_single_thread"] = {"value": sum(w.n * w.steps for w in ws) / d4, "cores": 1,
                               "seconds": d4,
                               "sample": "the first 32 of the 4096 instances, one after another"}
    w1 = W.w1_advection_square()
    r1c, d1c = scalar_rate(w1, w1.steps, False)
    res["w1_single_thread"] = {"value": r1c, "cores": 1, "seconds": d1c,
                               "sample": "the whole workload, 1024 cells x 1000 steps"}
    # served Sod: the first 8 requests of the seeded set with at most 2^12
    # cells, each solved in full (three components per cell-update)
    reqs = [r for r in W.w5_sod_requests(count=SERVE_COUNT, nmax=SERVE_NMAX) if r.n <= 1 << 12][:8]
    t0 = time.perf_counter()
    for r in reqs:
        op = O.Problem(O.EULER_ROE_EF, r.delta, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
        q = np.stack([O.quantise(r.U0[c], r.delta) for c in range(3)])
        O.step_euler(op, q, r.steps, omp=True)
    d5 = time.perf_counter() - t0
    res["w5_all_cores"] = {"value": sum(r.n * r.steps for r in reqs) / d5, "cores": omp_threads,
                           "seconds": d5,
                           "sample": f"{len(reqs)} Sod requests of at most 2^12 cells (the first "
                                     f"of the seeded set), each in full"}
    if level_state is not None:
        q = level_state
        t0 = time.perf_counter()
        O.entropy(q)
        t_e = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.level_transitions(q, q)
        O.row_defect(q, q)
        t_t = time.perf_counter() - t0
        res["levels_w2_ms"] = {"entropy": t_e * 1e3, "transitions_and_row_defect": t_t * 1e3}
    head = {"value": rA, "unit": "cell-updates/s", "cores": omp_threads, "kind": "oracle",
            "sample": f"burgers-eo 2^20 int32 cells x 10000 steps (the whole headline "
                      f"workload), OpenMP build of the C oracle on {omp_threads} threads, "
                      f"{dA:.1f} s, {model} ({avail} cores available); single thread: "
                      f"{r1:.3g} cell-updates/s on {s1} steps"}
    return head, res


def runtime_copy_rate(reps=5):
    """The HIP runtime's own device-to-device copy of 1 GiB (read + write bytes
    per second, HIP events): a reference point for the streaming kernels, not
    a ceiling (the library's one-step kernel streams faster)."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    t = float(np.median(ts))
    del a, b
    torch.cuda.empty_cache()
    return {"runtime_d2d_copy_GBps": 2.0 * n / t / 1e9,
            "frac_of_hbm_peak": 2.0 * n / t / 1e9 / HBM_PEAK_GBS}


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def copy_probe():
    import torch
    n = 256 << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "copies": 3}))


def run_extras_only(args, F, W, plans, stream, G):
    """Profiling aid: run one extra workload without the headline line."""
    extras = {}
    if args.only == "w3":
        w3 = W.w3_nyquist_advection(r=1e-3)
        p3 = F.make_problem(F.FLUX_UPWIND, w3.delta, w3.lam, w3.n, itype=F.I64, a=1.0)
        for tag, pl in (("stream", plans.STREAM_PLAN_W3), ("tblock", plans.BENCH_PLAN_W3)):
            S3 = Solver(F, p3, w3.u0, pl, stream)
            sec3, _ = time_solver(S3, w3.steps, max(args.steps, 1), args.warmup)
            S3.close()
            extras[f"w3_r0.001_{tag}"] = {"cell_updates_per_s": w3.n * w3.steps / sec3}
    elif args.only == "batch":
        extras.update(bench_batch(F, W, stream, G))
        extras.update(bench_tiled_mix(F, W, stream))
    elif args.only == "batch_only":
        extras.update(bench_batch_only(F, W, stream, reps=max(args.steps, 1)))
    elif args.only == "serve":
        extras.update(bench_serve(F, W, stream, G))
    elif args.only == "serve_closed":
        extras.update(bench_serve_closed(F, W, stream))
    elif args.only == "levels":
        extras.update(bench_levels(F, W, stream)[0])
    elif args.only == "nd":
        extras.update(bench_nd(F, W, plans, stream, G))
    elif args.only == "euler":
        extras.update(bench_euler(F, W, stream))
    elif args.only == "euler_cw":
        extras.update(bench_euler(F, W, stream, kinds=("componentwise",)))
    print(json.dumps({"extras": extras}), flush=True)


def time_plain(F, prob, u0, plan, steps, stream, reps=3):
    """Device time (HIP events on the library's stream) of `steps` steps of a
    fresh context per repetition; returns (seconds per solve, final state)."""
    import torch
    ts, q = [], None
    for rep in range(reps + 1):
        h = F.fqnm_create_from_field(prob, u0, stream)
        if plan is not None:
            F.fqnm_set_plan(h, *plan)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(torch.cuda.current_stream())
        F.fqnm_step(h, steps)
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
        if rep == reps:
            q = F.fqnm_get_state(h, prob)
        F.fqnm_destroy(h)
    return float(np.median(ts[1:])), q


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library drives one GPU; --gpus must be 1 "
              "(instances and grids shard across GPUs by design, but no multi-GPU path exists)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
        return
    from paper_2604_06947_amd import fqnm as F
    from paper_2604_06947_amd import plans
    from paper_2604_06947_amd import workloads as W

    stream = torch.cuda.current_stream().cuda_stream
    G = golden()
    out = {}
    extras = {}

    # ---------------- headline: Burgers EO LUT, 2^20 int32, 10000 steps -------------
    w = W.w2_burgers_step()
    if args.only not in ("", "w2"):
        return run_extras_only(args, F, W, plans, stream, G)
    prob = F.make_problem(F.FLUX_BURGERS_EO, w.delta, w.lam, w.n, itype=F.I32,
                          eval_=F.EVAL_LUT)
    log(f"[bench] W2 {w.name}")
    S = Solver(F, prob, w.u0, plans.BENCH_PLAN_W2, stream)
    sec, step_s = time_solver(S, w.steps, args.steps, args.warmup)
    inv = F.fqnm_invariants_get(S.h)
    w2_parity = parity("w2", S.cur.cpu().numpy(), G)
    q0_sum = S.q0_sum
    nl = S.launches(w.steps)
    plan = F.fqnm_get_plan(S.h)
    S.close()
    cu = w.n * w.steps
    value = cu / sec
    launch_s = step_s / nl
    units = w.n * plan["depth"] if plan["kernel"] != F.KERNEL_STREAM else w.n
    ops_tops = OPS_PER_CELL_UPDATE * units / launch_s / 1e12
    eff_gbs = 8.0 * units / launch_s / 1e9
    kname = {F.KERNEL_STREAM: "k_stream", F.KERNEL_TBLOCK: "k_tblock"}.get(plan["kernel"],
                                                                          f"kernel {plan['kernel']}")
    out.update({
        "metric": "cell-updates/s", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "burgers-eo-lut", "cells": w.n, "time_steps": w.steps,
                   "delta": w.delta, "cfl": 0.45, "state": "int32", "bc": "periodic",
                   "transfer": "Engquist-Osher, tabulated over [min q0, max q0]",
                   "plan": {"kernel": kname, "vec": plan["vec"], "depth": plan["depth"]}},
        "roofline": {
            "bound": "alu", "achieved": ops_tops, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": ops_tops / ALU_PEAK_TOPS,
            "ops_per_cell_update": OPS_PER_CELL_UPDATE,
            "cell_updates_per_launch": units, "avg_launch_us": launch_s * 1e6,
            "kernel": f"{kname}<int, P_LUT, {plan['vec']}>",
            "hbm_effective": {"bytes_per_cell_update": 8, "achieved_GBps": eff_gbs,
                              "frac_of_8TBps": eff_gbs / HBM_PEAK_GBS},
            **counter_fields(plans, "w2", launch_s)},
        "hbm_roofline_cell_updates_per_s": HBM_PEAK_GBS * 1e9 / 8.0,
        "conservation_ok": inv["sum"][0] == q0_sum,
        "parity_vs_oracle": w2_parity,
    })
    log(f"[bench] W2 {value:.4g} cell-updates/s, {sec*1e3:.2f} ms/solve, launch "
        f"{launch_s*1e6:.1f} us, parity {w2_parity}")

    if not args.no_extras:
        # ---------------- the first workload: latency of one small solve ------------
        w1 = W.w1_advection_square()
        p1 = F.make_problem(F.FLUX_UPWIND, w1.delta, w1.lam, w1.n, itype=F.I32, a=w1.a)
        t1, q1 = time_plain(F, p1, w1.u0, None, w1.steps, stream, reps=5)
        h1 = F.fqnm_create_from_field(p1, w1.u0, stream)
        pl1 = F.fqnm_get_plan(h1)  # the library's own choice for this grid
        F.fqnm_destroy(h1)
        extras["w1_latency"] = {"cells": w1.n, "time_steps": w1.steps, "us_per_solve": t1 * 1e6,
                                "cell_updates_per_s": w1.n * w1.steps / t1,
                                "plan": {"kernel": pl1["kernel"], "vec": pl1["vec"],
                                         "depth": pl1["depth"]},
                                "parity_vs_oracle": parity("w1", q1, G)}
        log(f"[bench] W1 {t1*1e6:.1f} us per solve")
        # ---------------- the headline workload at one step per pass ---------------
        ts, qs = time_plain(F, prob, w.u0, (F.KERNEL_STREAM, 4, 1), w.steps, stream, reps=2)
        g = 8.0 * w.n * w.steps / ts / 1e9
        extras["w2_stream_k1"] = {"kernel": "k_stream<int, P_LUT, 4>",
                                  "cell_updates_per_s": w.n * w.steps / ts,
                                  "avg_launch_us": ts / w.steps * 1e6, "achieved_GBps": g,
                                  "frac_of_hbm": g / HBM_PEAK_GBS,
                                  "parity_vs_oracle": parity("w2", qs, G)}
        log(f"[bench] W2 one step per pass: {w.n * w.steps / ts:.3e} cell-updates/s")

    # ---------------- extras: near-Nyquist int64 advection ------------------------------
    if not args.no_extras and args.only in ("", "w3"):
        extras.update(bench_w3(F, W, plans, stream, G))
    # ---------------- the FP64 finite-volume twin of the headline workload ----------
    if not args.no_extras and args.only in ("",):
        extras.update(bench_twin(F, W, plans, stream, value))
    # ---------------- batched: 4096 independent instances --------------------------
    if not args.no_extras and args.only in ("", "batch"):
        extras.update(bench_batch(F, W, stream, G))
        extras.update(bench_tiled_mix(F, W, stream))
    # ---------------- served: Sod requests with Poisson arrivals -----------------------
    if not args.no_extras and args.only in ("", "serve"):
        extras.update(bench_serve(F, W, stream, G))
    # ---------------- 2-D directional composition -------------------------------------
    if not args.no_extras and args.only in ("", "nd"):
        extras.update(bench_nd(F, W, plans, stream, G))
    # ---------------- single-grid Sod: componentwise and density-only -----------------
    if not args.no_extras and args.only in ("", "euler"):
        extras.update(bench_euler(F, W, stream))
    # ---------------- level statistics (entropy, transitions) -------------------------
    level_state = None
    if not args.no_extras and args.only in ("", "levels"):
        lv, level_state = bench_levels(F, W, stream)
        extras.update(lv)
    # ---------------- the runtime's device-to-device copy, for reference -------------
    if not args.no_extras and args.only in ("",):
        extras["runtime_copy"] = runtime_copy_rate()
    # ---------------- CPU oracle baseline --------------------------------------------
    if not args.no_cpu:
        head, detail = cpu_baseline(W, level_state)
        out["cpu_baseline"] = head
        extras["cpu_oracle"] = detail
    if extras:
        out["extras"] = extras
    print(json.dumps(out), flush=True)


def bench_w3(F, W, plans, stream, G):
    """Near-Nyquist advection, 2^24 int64 cells, 2000 steps, three delta/dx:
    the one-step streaming kernel (the honest HBM-bound figure, with its own
    roofline block) and the temporally blocked plan."""
    res = {}
    for r in (1e-2, 1e-3, 1e-4):
        w3 = W.w3_nyquist_advection(r=r)
        p3 = F.make_problem(F.FLUX_UPWIND, w3.delta, w3.lam, w3.n, itype=F.I64, a=1.0)
        for tag, pl in (("stream", plans.STREAM_PLAN_W3), ("tblock", plans.BENCH_PLAN_W3)):
            log(f"[bench] W3 r={r} {tag}")
            S3 = Solver(F, p3, w3.u0, pl, stream)
            sec3, st3 = time_solver(S3, w3.steps, 3, 1)
            nl3 = S3.launches(w3.steps)
            par3 = parity(f"w3_r{r:g}", S3.cur.cpu().numpy(), G)
            S3.close()
            d3 = pl[2] if pl[0] == F.KERNEL_TBLOCK else 1
            rate = w3.n * w3.steps / sec3
            ls = st3 / nl3
            ach3 = 16.0 * w3.n * d3 / ls / 1e9
            e = {"cell_updates_per_s": rate, "ms_per_solve": sec3 * 1e3, "avg_launch_us": ls * 1e6,
                 "kernel_GBps_algorithmic": ach3, "frac_of_hbm": ach3 / HBM_PEAK_GBS,
                 "frac_of_int64_roofline": rate / (HBM_PEAK_GBS * 1e9 / 16.0),
                 "parity_vs_oracle": par3}
            if tag == "stream":
                e["roofline"] = {"bound": "hbm", "achieved": ach3, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": ach3 / HBM_PEAK_GBS,
                                 "kernel": f"k_stream<long, P_UPWIND_POS, {pl[1]}>",
                                 "bytes_per_cell_update": 16,
                                 "algorithmic_bytes_per_launch": 16 * w3.n,
                                 **counter_fields(plans, "w3_stream", ls)}
            else:
                # many steps per HBM pass: the binding roof is VALU issue
                e["counters"] = {"kernel": f"k_tblock<long, P_UPWIND_POS, {pl[1]}>",
                                 **counter_fields(plans, "w3_tblock", ls)}
            res[f"w3_r{r:g}_{tag}"] = e
    return res


if __name__ == "__main__":
    main()
