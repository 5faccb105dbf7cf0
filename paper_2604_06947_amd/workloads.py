"""Seeded synthetic inputs for the FQNM hot path.

This module produces initial *fields* u0 (float64 point samples) and the
problem constants (delta, dt/dx, steps, boundary kind).  It holds none of the
method's arithmetic: quantisation, transfer maps and stepping happen on each
side (the HIP library and the CPU oracle) independently.  It imports neither.

Grid convention: cell centres x_i = i*dx, i = 0..N-1, dx = 1/N, on the
periodic unit interval (Sec. 2 places cell centres at x_i = i dx).

Workloads (all analytic initial data; the paper uses no dataset):
  W1  linear advection, N=1024, square wave on the closed interval [0.25, 0.5]
      plus 0.3 sin(2 pi x), delta=1e-4, dt/dx=0.5, 1000 steps, int32.
  W2  inviscid Burgers, N=2^20, u0 = 0.5 + sin(2 pi x) (the initial data of
      Sec. 3.2) plus a seeded step h*1[x >= xs], delta=1e-5, CFL 0.45,
      10000 steps, int32, Engquist-Osher transfer tabulated over the visited range.
  W3  near-Nyquist linear advection, N=2^24, u0 = cos(0.9 pi i) + 0.01 z_i,
      dt/dx=0.9, delta = r*dx for r in {1e-2, 1e-3, 1e-4}, 2000 steps, int64.
  W4  4096 independent instances (advection / Burgers 50:50), sizes
      log-uniform in [256, 65536], step counts uniform in [500, 5000], int32.
  W5  Sod-type Riemann problems for the Euler equations (gamma=1.4), states
      jittered +-20 % around Sod, sizes log-uniform in [2^10, 2^18], t=0.2.
  W6  2-D inviscid Burgers u_t + (u^2/2)_x + (u^2/2)_y = 0 (directional
      composition), periodic 4096 x 4096 (2^24 cells), u0 = 0.5 +
      sin(2 pi x) cos(2 pi y) plus a seeded step h*1[x >= xs], delta=1e-5,
      Engquist-Osher maps evaluated directly, dt/dx = dt/dy, summed CFL 0.45,
      1000 steps, int32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

UPWIND, BURGERS_EO, BURGERS_GODUNOV, LF_LINEAR, LF_BURGERS = 0, 1, 2, 3, 4
EULER_ROE, EULER_ROE_EF, BURGERS_MURMAN_ROE = 5, 6, 7
PERIODIC, OUTFLOW = 0, 1


@dataclass
class Scalar:
    """One scalar problem instance: flux kind and constants, the initial field
    and the number of steps.  ``width`` is the integer storage width."""
    kind: int
    delta: float
    lam: float
    u0: np.ndarray
    steps: int
    bc: int = PERIODIC
    width: int = 32
    a: float = 1.0
    alpha: float = 0.0
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.u0.size)


@dataclass
class Euler:
    """One Euler Riemann problem: conserved fields (rho, m, E) of shape (3, n)."""
    kind: int
    delta: float
    lam: float
    U0: np.ndarray
    steps: int
    bc: int = OUTFLOW
    gamma: float = 1.4
    left: tuple = (1.0, 0.0, 1.0)
    right: tuple = (0.125, 0.0, 0.1)
    t_final: float = 0.2
    name: str = ""

    @property
    def n(self):
        return int(self.U0.shape[1])


def grid(n):
    return np.arange(n, dtype=np.float64) / n


def w1_advection_square(n=1024, steps=1000):
    x = grid(n)
    u0 = ((x >= 0.25) & (x <= 0.5)).astype(np.float64) + 0.3 * np.sin(2 * np.pi * x)
    return Scalar(UPWIND, 1e-4, 0.5, u0, steps, PERIODIC, 32, a=1.0,
                  name=f"advection-square N={n} int32 upwind dt/dx=0.5 steps={steps}")


def burgers_cfl_lambda(u0, cfl):
    """dt/dx from the CFL number on the initial field: cfl / max|u0|."""
    return cfl / float(np.max(np.abs(u0)))


def w2_burgers_step(n=1 << 20, steps=10000, seed=2, cfl=0.45):
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.2, 1.0)
    xs = rng.uniform(0.0, 1.0)
    x = grid(n)
    u0 = 0.5 + np.sin(2 * np.pi * x) + h * (x >= xs)
    return Scalar(BURGERS_EO, 1e-5, burgers_cfl_lambda(u0, cfl), u0, steps, PERIODIC, 32,
                  name=f"burgers-eo-lut N={n} int32 delta=1e-5 cfl={cfl} steps={steps}",
                  extra={"h": h, "xs": xs})


def w3_nyquist_advection(r=1e-3, n=1 << 24, steps=2000, seed=3):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n)
    i = np.arange(n, dtype=np.float64)
    u0 = np.cos((0.9 * np.pi) * i) + 0.01 * z
    return Scalar(UPWIND, r / n, 0.9, u0, steps, PERIODIC, 64, a=1.0,
                  name=f"advection-nyquist N={n} int64 delta/dx={r} dt/dx=0.9 steps={steps}")


@dataclass
class Grid2D:
    """A 2-D scalar problem: field u0 of shape (ny, nx), x along the last axis."""
    kind: int
    delta: float
    lam: tuple  # (dt/dx, dt/dy)
    u0: np.ndarray
    steps: int
    bc: tuple = (PERIODIC, PERIODIC)
    width: int = 32
    a: tuple = (1.0, 1.0)
    alpha: tuple = (0.0, 0.0)
    name: str = ""

    @property
    def shape(self):
        return self.u0.shape


def w6_burgers_2d(nx=4096, ny=4096, steps=1000, seed=6, cfl=0.45, delta=1e-5):
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.2, 1.0)
    xs = rng.uniform(0.0, 1.0)
    x = grid(nx)[None, :]
    y = grid(ny)[:, None]
    u0 = 0.5 + np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + h * (x >= xs)
    lam = cfl / (2.0 * float(np.max(np.abs(u0))))  # the two directions share the CFL budget
    return Grid2D(BURGERS_EO, delta, (lam, lam), u0, steps,
                  name=f"burgers2d-eo {ny}x{nx} int32 delta={delta} cfl={cfl} steps={steps}")


def sine_step_field(x, b, A, m, theta, h, xs):
    return b + A * np.sin(2 * np.pi * m * x + theta) + h * (x >= xs)


def w4_batch(count=4096, seed=4, nmin=256, nmax=65536, smin=500, smax=5000, delta=1e-5):
    """Independent instances, drawn per instance in this order: kind, N, steps,
    b, A, m, theta, h, xs."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        adv = rng.uniform() < 0.5
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        steps = int(rng.integers(smin, smax + 1))
        b = rng.uniform(-0.25, 0.75)
        A = rng.uniform(0.2, 1.0)
        m = int(rng.integers(1, 4))
        theta = rng.uniform(0.0, 2 * np.pi)
        h = rng.uniform(0.2, 1.0)
        xs = rng.uniform(0.0, 1.0)
        u0 = sine_step_field(grid(n), b, A, m, theta, h, xs)
        if adv:
            s = Scalar(UPWIND, delta, 0.5, u0, steps, PERIODIC, 32, a=1.0, name=f"inst{k}-adv")
        else:
            s = Scalar(BURGERS_EO, delta, burgers_cfl_lambda(u0, 0.45), u0, steps, PERIODIC, 32,
                       name=f"inst{k}-burgers")
        s.extra = {"b": b, "A": A, "m": m, "theta": theta, "h": h, "xs": xs}
        out.append(s)
    return out


def w4_tiled_mix(count=192, seed=44, width=32, nmin=1 << 12, nmax=1 << 20, smin=500,
                 smax=2000, delta=1e-5):
    """Instances outside the batch's register-resident envelope (and a few
    inside it): the W4 families with sizes log-uniform in [nmin, nmax] (most
    above 65536 cells), every third one tabulated (eval LUT).  Drawn per
    instance in this order: kind, N, steps, b, A, m, theta, h, xs."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        adv = rng.uniform() < 0.5
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        steps = int(rng.integers(smin, smax + 1))
        b = rng.uniform(-0.25, 0.75)
        A = rng.uniform(0.2, 1.0)
        m = int(rng.integers(1, 4))
        theta = rng.uniform(0.0, 2 * np.pi)
        h = rng.uniform(0.2, 1.0)
        xs = rng.uniform(0.0, 1.0)
        u0 = sine_step_field(grid(n), b, A, m, theta, h, xs)
        if adv:
            s = Scalar(UPWIND, delta, 0.5, u0, steps, PERIODIC, width, a=1.0, name=f"mix{k}-adv")
        else:
            s = Scalar(BURGERS_EO, delta, burgers_cfl_lambda(u0, 0.45), u0, steps, PERIODIC, width,
                       name=f"mix{k}-burgers")
        s.extra = {"lut": k % 3 == 0}
        out.append(s)
    return out


# ---------------------------------------------------------------------------
# Euler / Sod
# ---------------------------------------------------------------------------
def sod_signal_speed_bound(left, right, gamma=1.4):
    """A closed-form upper estimate of the largest signal speed of a Riemann
    problem with states at rest or slow: max|u| + 2 max c of the two states.
    (For standard Sod: 2.37 against the exact 2.19.)"""
    cL = math.sqrt(gamma * left[2] / left[0])
    cR = math.sqrt(gamma * right[2] / right[0])
    return max(abs(left[1]), abs(right[1])) + 2.0 * max(cL, cR)


def sod_fields(n, left, right, gamma=1.4):
    """Conserved fields with the diaphragm between cells n/2-1 and n/2."""
    i = np.arange(n)
    isL = i < n // 2
    rho = np.where(isL, left[0], right[0]).astype(np.float64)
    u = np.where(isL, left[1], right[1]).astype(np.float64)
    p = np.where(isL, left[2], right[2]).astype(np.float64)
    m = rho * u
    E = p / (gamma - 1.0) + 0.5 * rho * u * u
    return np.stack([rho, m, E])


def sod_request(n, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), gamma=1.4, cfl=0.4,
                t_final=0.2, delta=1e-6, kind=EULER_ROE_EF, bc=OUTFLOW):
    """Fixed dt/dx per request: lam0 = cfl / S, steps = ceil(t/(lam0 dx)),
    then dt/dx = t / (steps dx) so that the final time is met exactly."""
    dx = 1.0 / n
    S = sod_signal_speed_bound(left, right, gamma)
    lam0 = cfl / S
    steps = int(math.ceil(t_final / (lam0 * dx)))
    lam = t_final / (steps * dx)
    return Euler(kind, delta, lam, sod_fields(n, left, right, gamma), steps, bc, gamma,
                 tuple(left), tuple(right), t_final, name=f"sod N={n}")


def w5_sod_requests(count=1000, seed=5, nmin=1 << 10, nmax=1 << 18, delta=1e-6):
    """Per request, drawn in this order: rhoL, pL, rhoR, pR jitter, N."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        rL = rng.uniform(0.8, 1.2)
        pL = rng.uniform(0.8, 1.2)
        rR = 0.125 * rng.uniform(0.8, 1.2)
        pR = 0.1 * rng.uniform(0.8, 1.2)
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        n += n & 1  # even, so that the diaphragm sits between cells n/2-1 and n/2
        out.append(sod_request(n, (rL, 0.0, pL), (rR, 0.0, pR), delta=delta))
    return out


def poisson_arrivals(count, rate, seed=55):
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


# ---------------------------------------------------------------------------
# Small random inputs for parity and property tests
# ---------------------------------------------------------------------------
def random_states(n, lo, hi, seed):
    """Uniform random integer states in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=n, dtype=np.int64)


def random_smooth_step(n, seed, b=0.5, amp=1.0):
    """A seeded smooth-plus-step field (the W4 family) on n cells."""
    rng = np.random.default_rng(seed)
    A = amp * rng.uniform(0.2, 1.0)
    m = int(rng.integers(1, 4))
    theta = rng.uniform(0.0, 2 * np.pi)
    h = rng.uniform(0.2, 1.0)
    xs = rng.uniform(0.0, 1.0)
    return sine_step_field(grid(n), b, A, m, theta, h, xs)
