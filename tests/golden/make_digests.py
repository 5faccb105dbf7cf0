"""Write tests/golden/full_size_digests.txt: SHA-256 digests of the oracle's
final integer states on the benchmarked workloads at their full sizes.

This script calls only the oracle (``oracle/``) and the seeded input
generators (``paper_2604_06947_amd/workloads.py``, which hold no arithmetic
of the method).  The GPU tests compare the digests of the device states with
these lines, so every benchmarked workload has an element-by-element parity
check at full size without storing the states themselves.

Digest of a state: SHA-256 of its values as little-endian int64, the three
Euler components (rho, m, E) one after the other.  Each line:

    key  n  steps  sum  sha256

``sum`` is the exact sum of the integers of the first component (a second
check that can say "mass differs" when a digest does not match).

Workloads (names as in workloads.py):
  w1                     advection square wave, 1024 cells x 1000 steps, int32
  w2                     Burgers EO, 2^20 int32 cells x 10000 steps
  w3_r<r>                near-Nyquist advection, 2^24 int64 cells x 2000 steps,
                         r = delta/dx in {1e-2, 1e-3, 1e-4}
  w6                     2-D Burgers EO, 4096 x 4096 int32 cells x 1000 steps
  w4_<k>                 every one of the 4096 batch instances
  w5_<i>                 the served Sod requests (1000, sizes 2^10..2^18)
                         with n <= 16384, plus the largest request and 7
                         more larger ones drawn with seed 505

Usage: python tests/golden/make_digests.py [--only w2,w4,...] [--threads T]
Existing lines of the other keys are kept.  The full set takes roughly
half an hour on 8 host cores.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "full_size_digests.txt")
W5_SMALL_MAX = 16384
W5_LARGE_SEED = 505
W5_LARGE_COUNT = 8


def digest(q) -> str:
    return hashlib.sha256(np.ascontiguousarray(q, dtype="<i8").tobytes()).hexdigest()


def line(key, n, steps, q):
    first = np.asarray(q).reshape(-1) if np.asarray(q).ndim == 1 else np.asarray(q)[0]
    return f"{key} {n} {steps} {int(np.asarray(first, dtype=np.int64).sum())} {digest(q)}"


def w5_selected(reqs):
    """Indices of the requests with expected digests: every request of at most
    W5_SMALL_MAX cells, the largest one, and W5_LARGE_COUNT - 1 more of the
    larger ones drawn with a seeded generator."""
    ns = np.array([r.n for r in reqs])
    small = [int(i) for i in np.nonzero(ns <= W5_SMALL_MAX)[0]]
    large = [int(i) for i in np.nonzero(ns > W5_SMALL_MAX)[0]]
    top = int(np.argmax(ns))
    rest = [i for i in large if i != top]
    rng = np.random.default_rng(W5_LARGE_SEED)
    pick = sorted(int(i) for i in rng.choice(rest, size=W5_LARGE_COUNT - 1, replace=False))
    return small, [top] + pick


def run(only, threads):
    import oracle as O
    from paper_2604_06947_amd import workloads as W

    out = {}
    t0 = time.time()

    def log(*a):
        print(f"[{time.time() - t0:7.1f}s]", *a, flush=True)

    def scalar(w, omp):
        p = O.Problem(w.kind, w.delta, w.lam, bc=w.bc, width=w.width, a=w.a, alpha=w.alpha)
        return O.step(p, O.quantise(w.u0, w.delta, w.width), w.steps, omp=omp)

    if "w1" in only:
        w = W.w1_advection_square()
        out["w1"] = line("w1", w.n, w.steps, scalar(w, False))
        log("w1")
    if "w2" in only:
        w = W.w2_burgers_step()
        out["w2"] = line("w2", w.n, w.steps, scalar(w, True))
        log("w2")
    if "w3" in only:
        for r in (1e-2, 1e-3, 1e-4):
            w = W.w3_nyquist_advection(r=r)
            k = f"w3_r{r:g}"
            out[k] = line(k, w.n, w.steps, scalar(w, True))
            log(k)
    if "w6" in only:
        w = W.w6_burgers_2d()
        axes = [O.Problem(w.kind, w.delta, w.lam[0], bc=w.bc[0], width=w.width, a=w.a[0]),
                O.Problem(w.kind, w.delta, w.lam[1], bc=w.bc[1], width=w.width, a=w.a[1])]
        q = O.step_nd(axes, O.quantise(w.u0, w.delta, w.width), w.steps, omp=True)
        out["w6"] = line("w6", q.size, w.steps, q.reshape(-1))
        log("w6")
    if "w4" in only:
        ws = W.w4_batch()

        def one(k):
            return f"w4_{k}", line(f"w4_{k}", ws[k].n, ws[k].steps, scalar(ws[k], False))

        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            for k, v in ex.map(one, range(len(ws))):
                out[k] = v
        log("w4")
    if "w5" in only:
        reqs = W.w5_sod_requests()
        small, large = w5_selected(reqs)

        def one(i, omp=False):
            r = reqs[i]
            p = O.Problem(r.kind, r.delta, r.lam, bc=r.bc, gamma=r.gamma)
            q0 = np.stack([O.quantise(r.U0[c], r.delta) for c in range(3)])
            return f"w5_{i}", line(f"w5_{i}", r.n, r.steps, O.step_euler(p, q0, r.steps, omp=omp))

        order = sorted(small, key=lambda i: -reqs[i].n)  # longest first
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            for k, v in ex.map(one, order):
                out[k] = v
        log("w5 small", len(small))
        for i in large:
            k, v = one(i, omp=True)
            out[k] = v
            log(k, reqs[i].n, reqs[i].steps)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="w1,w2,w3,w6,w4,w5")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", str(a.threads))
    only = set(a.only.split(","))
    lines = {}
    if os.path.exists(OUT):
        for l in open(OUT):
            if l.strip() and not l.startswith("#"):
                lines[l.split()[0]] = l.rstrip("\n")
    lines.update(run(only, a.threads))

    def order(k):
        base, _, idx = k.partition("_")
        return (base, int(idx) if idx.isdigit() else 0, k)

    with open(OUT + ".tmp", "w") as f:
        f.write("# key n steps sum(first component) sha256(final state as <i8)\n")
        f.write("# written by tests/golden/make_digests.py from the oracle; do not edit\n")
        for k in sorted(lines, key=order):
            f.write(lines[k] + "\n")
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
