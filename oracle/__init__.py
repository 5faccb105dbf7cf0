"""CPU oracle for the FQNM integer-transfer hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or runs anything here, and nothing
here imports the product package.

Contents
--------
* ``fqnm_oracle.c`` -- C reference stepper (quantisation, the transfer maps
  of every flux kind, the Jacobi integer update, invariants, the FP64
  classical comparators, the Euler/Roe transfer and level statistics).
  Compiled with gcc, contraction off, by :func:`build`: once plain
  (single-threaded) and once with OpenMP (the same integers; for the
  full-size digests and the all-cores CPU baseline).
* :mod:`oracle.exact` -- exact solutions used as independent references
  (exact shift, Hopf-Lax/Lax-Oleinik for Burgers, exact Riemann solver).

Every function cites the passage of the paper it follows (arXiv 2604.06947).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fqnm_oracle.c")
LIB = os.path.join(HERE, "liboracle_fqnm.so")
# The same source built with -fopenmp: the stepping loops run over cells (or
# interfaces) that read only the state before the step, so the integers are
# those of the plain build; it times the all-cores CPU baseline and writes the
# full-size expected digests in minutes instead of hours.
LIB_OMP = os.path.join(HERE, "liboracle_fqnm_omp.so")

# Flux kinds and boundary kinds: the numbering of the public interface.
UPWIND, BURGERS_EO, BURGERS_GODUNOV, LF_LINEAR, LF_BURGERS = 0, 1, 2, 3, 4
EULER_ROE, EULER_ROE_EF, BURGERS_MURMAN_ROE = 5, 6, 7
PERIODIC, OUTFLOW = 0, 1

STATUS = {0: "ok", 1: "bad argument", 2: "integer range exceeded", 3: "non-finite value"}


class OracleError(RuntimeError):
    pass


class _Problem(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("bc", C.c_int32), ("width", C.c_int32), ("pad_", C.c_int32),
        ("a", C.c_double), ("alpha", C.c_double), ("gamma", C.c_double),
        ("delta", C.c_double), ("lambda_", C.c_double),
    ]


def _stale(path):
    return not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (contraction off, no fast-math), once plain
    (single-threaded) and once with OpenMP."""
    for path, extra in ((LIB, ["-Wno-unknown-pragmas"]), (LIB_OMP, ["-fopenmp"])):
        if force or _stale(path):
            tmp = path + ".tmp"
            subprocess.check_call([
                "gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                "-shared", "-Wall"] + extra + ["-o", tmp, SRC, "-lm"])
            os.replace(tmp, path)
    return LIB


_libs = {}


def lib(omp: bool = False):
    """The plain single-threaded oracle, or (omp=True) the OpenMP build of the
    same source."""
    path = LIB_OMP if omp else LIB
    if path not in _libs:
        if _stale(LIB) or _stale(LIB_OMP):
            build(force=True)
        L = C.CDLL(path)
        P = C.POINTER(_Problem)
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.ofq_step.argtypes = [P, C.c_int64, i64p, C.c_int64, C.POINTER(C.c_int64)]
        L.ofq_step.restype = C.c_int
        L.ofq_quantise.argtypes = [f64p, C.c_int64, C.c_double, C.c_int32, i64p]
        L.ofq_quantise.restype = C.c_int
        L.ofq_reconstruct.argtypes = [i64p, C.c_int64, C.c_double, f64p]
        L.ofq_reconstruct.restype = None
        L.ofq_phi.argtypes = [P, C.c_int32, C.c_int64, C.POINTER(C.c_int64)]
        L.ofq_phi.restype = C.c_int
        L.ofq_interface_flux.argtypes = [P, C.c_int64, C.c_int64, C.POINTER(C.c_int64)]
        L.ofq_interface_flux.restype = C.c_int
        L.ofq_invariants.argtypes = [i64p, C.c_int64, C.c_int32] + [C.c_void_p] * 6
        L.ofq_invariants.restype = None
        L.ofq_classical_flux.argtypes = [P, C.c_double, C.c_double]
        L.ofq_classical_flux.restype = C.c_double
        L.ofq_classical_step.argtypes = [P, C.c_int64, f64p, C.c_int64]
        L.ofq_classical_step.restype = C.c_int
        L.ofq_step_euler.argtypes = [P, C.c_int64, i64p, i64p, i64p, C.c_int64, i64p]
        L.ofq_step_euler.restype = C.c_int
        L.ofq_euler_flux.argtypes = [P, i64p, i64p, f64p, f64p]
        L.ofq_euler_flux.restype = C.c_int
        L.ofq_classical_step_euler.argtypes = [P, C.c_int64, f64p, f64p, f64p, C.c_int64]
        L.ofq_classical_step_euler.restype = C.c_int
        L.ofq_level_histogram.argtypes = [i64p, C.c_int64, i64p, i64p]
        L.ofq_level_histogram.restype = C.c_int64
        L.ofq_entropy.argtypes = [i64p, C.c_int64]
        L.ofq_entropy.restype = C.c_double
        L.ofq_level_transitions.argtypes = [i64p, i64p, C.c_int64, i64p, i64p, i64p]
        L.ofq_level_transitions.restype = C.c_int64
        L.ofq_step_euler_density.argtypes = [P, C.c_int64, i64p, f64p, f64p, C.c_int64,
                                             C.POINTER(C.c_int64)]
        L.ofq_step_euler_density.restype = C.c_int
        L.ofq_step_nd.argtypes = [C.POINTER(_Problem), C.c_int32, i64p, i64p, C.c_int64,
                                  C.POINTER(C.c_int64)]
        L.ofq_step_nd.restype = C.c_int
        L.ofq_row_defect.argtypes = [i64p, i64p, C.c_int64]
        L.ofq_row_defect.restype = C.c_double
        L.ofq_threads.argtypes = []
        L.ofq_threads.restype = C.c_int
        _libs[path] = L
    return _libs[path]


def threads(omp: bool = False) -> int:
    """Threads the stepping loops of that build use (1 for the plain build)."""
    return int(lib(omp).ofq_threads())


class Problem:
    """Scalar or Euler problem as the paper states it: flux kind, delta, dt/dx,
    boundary kind, plus the kind's own constants (a, alpha, gamma)."""

    def __init__(self, kind, delta, lam, bc=PERIODIC, width=64, a=1.0, alpha=0.0, gamma=1.4):
        self.kind, self.delta, self.lam, self.bc, self.width = kind, delta, lam, bc, width
        self.a, self.alpha, self.gamma = a, alpha, gamma

    def c(self) -> _Problem:
        return _Problem(self.kind, self.bc, self.width, 0, self.a, self.alpha, self.gamma,
                        self.delta, self.lam)


def _check(st):
    if st != 0:
        raise OracleError(STATUS.get(st, f"status {st}"))


def quantise(u, delta, width=64):
    """eq:quantisation: q = rint(u / delta) (IEEE division, half-to-even)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    q = np.empty(u.shape, np.int64)
    _check(lib().ofq_quantise(u, u.size, float(delta), int(width), q))
    return q


def reconstruct(q, delta):
    """eq:reconstruction_operator: u = delta * q."""
    q = np.ascontiguousarray(q, dtype=np.int64)
    u = np.empty(q.shape, np.float64)
    lib().ofq_reconstruct(q, q.size, float(delta), u)
    return u


def step(prob: Problem, q, nsteps, return_ledger=False, omp=False):
    """nsteps Jacobi steps of eq:update_rule_conservative_form; returns a copy."""
    q = np.array(q, dtype=np.int64, copy=True)
    led = C.c_int64(0)
    _check(lib(omp).ofq_step(C.byref(prob.c()), q.size, q, int(nsteps), C.byref(led)))
    return (q, led.value) if return_ledger else q


def step_nd(axes, q, nsteps, return_ledger=False, omp=False):
    """d-dimensional directional composition (Thm dimension_extension).

    ``q`` is a C-ordered array whose LAST numpy axis is the contiguous one;
    ``axes[m]`` is the Problem of direction m, with ``axes[0]`` for that last
    numpy axis, ``axes[1]`` for the one before it, and so on."""
    q = np.array(q, dtype=np.int64, copy=True, order="C")
    dim = q.ndim
    assert len(axes) == dim and 1 <= dim <= 3
    shape = np.array(q.shape[::-1], dtype=np.int64)
    arr = (_Problem * dim)(*[a.c() for a in axes])
    led = C.c_int64(0)
    flat = q.reshape(-1)
    _check(lib(omp).ofq_step_nd(arr, dim, shape, flat, int(nsteps), C.byref(led)))
    q = flat.reshape(q.shape)
    return (q, led.value) if return_ledger else q


def trajectory(prob: Problem, q, nsteps):
    """All states q^0..q^nsteps as a (nsteps+1, n) array."""
    out = [np.array(q, dtype=np.int64)]
    for _ in range(nsteps):
        out.append(step(prob, out[-1], 1))
    return np.stack(out)


def phi(prob: Problem, plus: bool, q: int) -> int:
    """eq:flux_table for one state."""
    out = C.c_int64(0)
    _check(lib().ofq_phi(C.byref(prob.c()), 1 if plus else 0, int(q), C.byref(out)))
    return out.value


def interface_flux(prob: Problem, qL: int, qR: int) -> int:
    """eq:numerical_count_flux_definition (split) or the two-point rule."""
    out = C.c_int64(0)
    _check(lib().ofq_interface_flux(C.byref(prob.c()), int(qL), int(qR), C.byref(out)))
    return out.value


def invariants(q, periodic=True):
    """Exact sum, min, max and total variation (with the periodic wrap term)."""
    q = np.ascontiguousarray(q, dtype=np.int64)
    sh, sl, mn, mx, th, tl = (C.c_int64(), C.c_uint64(), C.c_int64(), C.c_int64(),
                              C.c_int64(), C.c_uint64())
    lib().ofq_invariants(q, q.size, 1 if periodic else 0, C.byref(sh), C.byref(sl),
                         C.byref(mn), C.byref(mx), C.byref(th), C.byref(tl))
    return {"sum": (sh.value << 64) + sl.value, "min": mn.value, "max": mx.value,
            "tv": (th.value << 64) + tl.value}


def classical_flux(prob: Problem, uL: float, uR: float) -> float:
    """eq:classical_operator_definition: F(uL,uR) = f+(uL) + f-(uR) in FP64."""
    return lib().ofq_classical_flux(C.byref(prob.c()), float(uL), float(uR))


def classical_step(prob: Problem, u, nsteps):
    """FP64 split finite-volume scheme u <- u - lambda (F_R - F_L)."""
    u = np.array(u, dtype=np.float64, copy=True)
    _check(lib().ofq_classical_step(C.byref(prob.c()), u.size, u, int(nsteps)))
    return u


def step_euler(prob: Problem, q3, nsteps, return_ledger=False, omp=False):
    """Componentwise quantised Roe transfer for the Euler system (Sec. 3.3).
    q3 has shape (3, n): rho, m, E counts."""
    q3 = np.array(q3, dtype=np.int64, copy=True)
    r, m, E = (np.ascontiguousarray(q3[c]) for c in range(3))
    led = np.zeros(3, np.int64)
    _check(lib(omp).ofq_step_euler(C.byref(prob.c()), r.size, r, m, E, int(nsteps), led))
    out = np.stack([r, m, E])
    return (out, led) if return_ledger else out


def step_euler_density(prob: Problem, qr, m, E, nsteps, return_ledger=False):
    """Density-only quantised Roe update (Sec. 3.3): integer density counts qr,
    real momentum m and energy E.  Returns (qr, m, E) [, density ledger]."""
    qr = np.array(qr, dtype=np.int64, copy=True)
    m = np.array(m, dtype=np.float64, copy=True)
    E = np.array(E, dtype=np.float64, copy=True)
    led = C.c_int64(0)
    _check(lib().ofq_step_euler_density(C.byref(prob.c()), qr.size, qr, m, E, int(nsteps),
                                        C.byref(led)))
    return (qr, m, E, led.value) if return_ledger else (qr, m, E)


def euler_flux(prob: Problem, qL, qR):
    """FP64 Roe flux of two integer states and its wave decomposition
    (ub, Hb, cb, c2, a1, a2, a3, l1, l2, l3)."""
    F = np.zeros(3)
    w = np.zeros(10)
    _check(lib().ofq_euler_flux(C.byref(prob.c()), np.asarray(qL, np.int64),
                                np.asarray(qR, np.int64), F, w))
    return F, w


def classical_step_euler(prob: Problem, U, nsteps):
    """FP64 Roe finite-volume trajectory on conserved variables, shape (3, n)."""
    U = np.array(U, dtype=np.float64, copy=True)
    r, m, E = (np.ascontiguousarray(U[c]) for c in range(3))
    _check(lib().ofq_classical_step_euler(C.byref(prob.c()), r.size, r, m, E, int(nsteps)))
    return np.stack([r, m, E])


def level_histogram(q):
    """Occupied levels k and counts c_k (Supplementary Information, eq:pk_definition)."""
    q = np.ascontiguousarray(q, dtype=np.int64)
    lv = np.empty(q.size, np.int64)
    ct = np.empty(q.size, np.int64)
    m = lib().ofq_level_histogram(q, q.size, lv, ct)
    return lv[:m].copy(), ct[:m].copy()


def entropy(q) -> float:
    """eq:discrete_entropy: S = -sum_k p_k log p_k."""
    q = np.ascontiguousarray(q, dtype=np.int64)
    return lib().ofq_entropy(q, q.size)


def level_transitions(q0, q1):
    """Sorted (k, k', N_{k'k}) triples of the one-step level-transition counts."""
    q0 = np.ascontiguousarray(q0, dtype=np.int64)
    q1 = np.ascontiguousarray(q1, dtype=np.int64)
    f = np.empty(q0.size, np.int64)
    t = np.empty(q0.size, np.int64)
    c = np.empty(q0.size, np.int64)
    m = lib().ofq_level_transitions(q0, q1, q0.size, f, t, c)
    return f[:m].copy(), t[:m].copy(), c[:m].copy()


def row_defect(q0, q1) -> float:
    """rho = max_k' |sum_k N_{k'k}/c_k - 1| over the levels occupied in q1
    (Supplementary Information, eq:empirical_M, Remark doubly_stochastic_condition)."""
    q0 = np.ascontiguousarray(q0, dtype=np.int64)
    q1 = np.ascontiguousarray(q1, dtype=np.int64)
    assert q0.size == q1.size
    return lib().ofq_row_defect(q0, q1, q0.size)
