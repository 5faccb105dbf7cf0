"""Pins of the oracle's FP64 classical comparators, its invariants and its
OpenMP build -- none of them compares a function with itself.

* ``classical_step`` (Sec. 2.1, eq:classical_operator_definition): exact
  one-cell shifts at unit Courant number, an exact-rational stepper on dyadic
  data (where every FP64 operation is exact), the per-step correspondence with
  the quantised update (Prop. operator_quantisation_error) and the outflow
  mass balance.
* ``classical_step_euler`` (the FP64 Roe trajectory of Sec. 3.3): constant
  states are fixed, fully supersonic data is pure upwinding of the physical
  flux (written here from the Euler equations, not from the Roe average),
  and the error against the exact Riemann solution falls with N.
* ``invariants``: hand-worked total variations with and without the periodic
  wrap term, including 128-bit sums.
* The literal operation order of eq:flux_table against the canonical one
  (negative control (ii) of Thm transfer_operator_equivalence).
* The OpenMP build of the oracle against the plain build.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle import exact as X
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------------------
# classical_step at unit Courant number: an exact one-cell shift (dyadic data,
# so every subtraction is exact)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("a", [1.0, -1.0])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW])
def test_classical_unit_courant_shift(a, bc):
    rng = np.random.default_rng(41)
    n = 29
    u0 = rng.integers(-1000, 1001, size=n).astype(np.float64) * 2.0 ** -10
    p = O.Problem(O.UPWIND, 1.0, 1.0, bc=bc, a=a)
    u1 = O.classical_step(p, u0, 1)
    if bc == O.PERIODIC:
        assert np.array_equal(u1, np.roll(u0, 1 if a > 0 else -1))
        assert np.array_equal(O.classical_step(p, u0, n), u0)  # n shifts: identity
    elif a > 0:  # inflow at the left end copies cell 0 into its ghost
        assert np.array_equal(u1, np.concatenate([u0[:1], u0[:-1]]))
    else:
        assert np.array_equal(u1, np.concatenate([u0[1:], u0[-1:]]))


# ---------------------------------------------------------------------------
# classical_step on dyadic data against exact rational arithmetic.  The
# stepper below is eq:classical_operator_definition with the splittings of
# eq:flux_splitting (and the two-point Burgers fluxes) in Fraction arithmetic;
# on these inputs every FP64 operation of the oracle is exact, so the two must
# agree bit for bit.
# ---------------------------------------------------------------------------
def frac_flux(kind, a, alpha):
    f = (lambda u: a * u) if kind in (O.UPWIND, O.LF_LINEAR) else (lambda u: u * u / 2)

    def fp(u):
        if kind == O.UPWIND:
            return max(a, 0) * u
        if kind == O.BURGERS_EO:
            return max(u, 0) ** 2 / 2
        return (f(u) + alpha * u) / 2

    def fm(u):
        if kind == O.UPWIND:
            return min(a, 0) * u
        if kind == O.BURGERS_EO:
            return min(u, 0) ** 2 / 2
        return (f(u) - alpha * u) / 2

    def F(uL, uR):
        if kind == O.BURGERS_MURMAN_ROE:
            return f(uL) if uL + uR >= 0 else f(uR)
        if kind == O.BURGERS_GODUNOV:
            if uL <= uR:  # minimum of f over [uL, uR]
                return 0 if uL <= 0 <= uR else min(f(uL), f(uR))
            return max(f(uL), f(uR))  # maximum of f over [uR, uL]
        return fp(uL) + fm(uR)

    return F


def frac_classical_step(F, lam, u, bc):
    n = len(u)
    if bc == O.PERIODIC:
        G = [F(u[i - 1], u[i]) for i in range(n)] + [F(u[n - 1], u[0])]
    else:
        G = [F(u[0], u[0])] + [F(u[i - 1], u[i]) for i in range(1, n)] + [F(u[n - 1], u[n - 1])]
    return [u[i] - lam * (G[i + 1] - G[i]) for i in range(n)]


CLASSICAL = [  # kind, lambda, a, alpha, steps kept exact in 53 bits
    (O.UPWIND, Fraction(1, 2), Fraction(1), Fraction(0), 10),
    (O.UPWIND, Fraction(3, 4), Fraction(-1), Fraction(0), 8),
    (O.UPWIND, Fraction(1, 4), Fraction(3, 4), Fraction(0), 8),
    (O.LF_LINEAR, Fraction(1, 4), Fraction(1, 2), Fraction(1), 8),
    (O.BURGERS_EO, Fraction(1, 4), Fraction(1), Fraction(0), 2),
    (O.BURGERS_GODUNOV, Fraction(1, 2), Fraction(1), Fraction(0), 2),
    (O.BURGERS_MURMAN_ROE, Fraction(1, 4), Fraction(1), Fraction(0), 2),
    (O.LF_BURGERS, Fraction(1, 4), Fraction(1), Fraction(2), 2),
]


@pytest.mark.parametrize("kind,lam,a,alpha,steps", CLASSICAL)
@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW])
def test_classical_step_exact_rational(kind, lam, a, alpha, steps, bc):
    F = frac_flux(kind, a, alpha)
    p = O.Problem(kind, 1.0, float(lam), bc=bc, a=float(a), alpha=float(alpha))
    rng = np.random.default_rng(43)
    cases = [list(t) for t in itertools.product(range(-3, 4), repeat=2)]
    cases += [list(rng.integers(-64, 65, size=n)) for n in (1, 3, 5, 8) for _ in range(40)]
    for k in cases:
        ref = [Fraction(int(v), 64) for v in k]
        got = np.array([float(v) for v in ref])
        for _ in range(steps):
            ref = frac_classical_step(F, lam, ref, bc)
            assert all(Fraction(float(v)) == v for v in ref), "inputs left the exact range"
            got = O.classical_step(p, got, 1)
            assert [Fraction(float(v)) for v in got] == ref, (kind, k)


# ---------------------------------------------------------------------------
# Prop. operator_quantisation_error through classical_step itself: one
# classical step from the reconstructed state delta*q^n differs from the
# reconstructed quantised step delta*q^{n+1} by at most 2 delta per cell for
# split kinds (four roundings of at most 1/2) and delta for two-point kinds.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,kw,bound", [
    (O.UPWIND, dict(a=1.0), 2), (O.UPWIND, dict(a=-0.6), 2), (O.BURGERS_EO, {}, 2),
    (O.LF_BURGERS, dict(alpha=1.8), 2), (O.BURGERS_GODUNOV, {}, 1),
    (O.BURGERS_MURMAN_ROE, {}, 1)])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW])
def test_classical_step_tracks_quantised_step(kind, kw, bound, bc):
    n, delta = 300, 1e-5
    u0 = W.random_smooth_step(n, seed=53, b=0.2)
    lam = 0.4 / float(np.max(np.abs(u0)))
    if kind == O.UPWIND:
        lam = 0.7
    if kind == O.LF_BURGERS:
        lam = 0.5 / kw["alpha"]
    p = O.Problem(kind, delta, lam, bc=bc, **kw)
    q = O.quantise(u0, delta)
    worst = 0.0
    for _ in range(30):
        q1 = O.step(p, q, 1)
        u = O.reconstruct(q, delta)
        cl = O.classical_step(p, u, 1)
        res = np.abs(O.reconstruct(q1, delta) - cl)
        eps = 64 * 2.0 ** -53 * (np.abs(u) + 4.0)
        assert np.all(res <= bound * delta + eps), (kind, float(np.max(res / delta)))
        worst = max(worst, float(np.max(res / delta)))
        q = q1
    assert worst > 0.25 * bound  # not vacuous


# ---------------------------------------------------------------------------
# Outflow mass balance of classical_step: sum(u^{n+1}) - sum(u^n) equals
# lambda*(F(u_0,u_0) - F(u_{N-1},u_{N-1})) exactly on dyadic data (the sums
# are taken exactly; the interface terms telescope).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,a", [(O.UPWIND, 1.0), (O.UPWIND, -1.0), (O.BURGERS_EO, 1.0),
                                    (O.BURGERS_GODUNOV, 1.0)])
def test_classical_outflow_mass_balance(kind, a):
    F = frac_flux(kind, Fraction(a), Fraction(0))
    lam = Fraction(1, 4)
    p = O.Problem(kind, 1.0, float(lam), bc=O.OUTFLOW, a=a)
    rng = np.random.default_rng(47)
    for _ in range(30):
        u = rng.integers(-64, 65, size=9).astype(np.float64) / 64.0
        u1 = O.classical_step(p, u, 1)
        uf = [Fraction(v) for v in u]
        lhs = sum(Fraction(v) for v in u1) - sum(uf)
        rhs = lam * (F(uf[0], uf[0]) - F(uf[-1], uf[-1]))
        assert lhs == rhs


# ---------------------------------------------------------------------------
# classical_step_euler (FP64 Roe scheme on conserved variables, Sec. 3.3)
# ---------------------------------------------------------------------------
def conserved(rho, u, p, gamma=1.4):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def euler_flux_exact(U, gamma=1.4):
    """Physical flux of the 1-D Euler equations (mass, momentum, energy)."""
    rho, m, E = U
    u = m / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * u * u)
    return np.stack([m, m * u + p, u * (E + p)])


@pytest.mark.parametrize("kind", [O.EULER_ROE, O.EULER_ROE_EF])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW])
def test_classical_euler_constant_state_fixed(kind, bc):
    p = O.Problem(kind, 1.0, 0.3, bc=bc, gamma=1.4)
    for rho, u, pr in [(1.0, 0.0, 1.0), (0.3, -0.7, 0.2), (2.5, 1.9, 0.8)]:
        U = conserved(np.full(17, rho), np.full(17, u), np.full(17, pr))
        assert np.array_equal(O.classical_step_euler(p, U, 5), U)


@pytest.mark.parametrize("kind", [O.EULER_ROE, O.EULER_ROE_EF])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_classical_euler_supersonic_is_upwind(kind, sign):
    """Where every state moves faster than its sound speed in one direction,
    all three Roe waves travel that way and the flux is the physical flux of
    the upwind cell: one step is u_i - lambda*(f(U_i) - f(U_{i-1})) (or the
    mirror image), with outflow ghosts copying the end cells."""
    rng = np.random.default_rng(59)
    n, lam = 40, 0.1
    rho = rng.uniform(0.8, 1.2, n)
    u = sign * rng.uniform(3.0, 3.5, n)
    pr = rng.uniform(0.5, 0.9, n)  # c <= sqrt(1.4*0.9/0.8) < 1.3 < |u|
    U = conserved(rho, u, pr)
    p = O.Problem(kind, 1.0, lam, bc=O.OUTFLOW, gamma=1.4)
    got = O.classical_step_euler(p, U, 1)
    f = euler_flux_exact(U)
    if sign > 0:
        fl = np.concatenate([f[:, :1], f[:, :-1]], axis=1)  # flux through the left face
        ref = U - lam * (f - fl)
    else:
        fr = np.concatenate([f[:, 1:], f[:, -1:]], axis=1)  # flux through the right face
        ref = U - lam * (fr - f)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_classical_euler_converges_to_exact_riemann():
    errs = []
    for n in (128, 256, 512):
        r = W.sod_request(n)
        p = O.Problem(r.kind, 1.0, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
        U = O.classical_step_euler(p, r.U0, r.steps)
        x = W.grid(n)
        xd = (n // 2 - 0.5) / n
        ref, _, _ = X.riemann_exact(r.left, r.right, (x - xd) / r.t_final)
        errs.append(float(np.mean(np.abs(U[0] - ref))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.02


def test_classical_euler_mirror_symmetry():
    """x -> -x maps (rho, m, E)_i to (rho, -m, E)_{N-1-i}; the scheme commutes
    with it up to the rounding of reordered sums."""
    r = W.sod_request(200, left=(1.1, 0.3, 0.9), right=(0.2, -0.1, 0.15))
    p = O.Problem(r.kind, 1.0, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
    M = np.array([1.0, -1.0, 1.0])[:, None]
    a = O.classical_step_euler(p, r.U0, 60)
    b = O.classical_step_euler(p, (M * r.U0)[:, ::-1].copy(), 60)
    assert np.allclose((M * b)[:, ::-1], a, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------
# invariants: total variation with and without the periodic wrap term (the
# reading of Lemma cfl_monotone (ii) on a periodic grid), exact 128-bit sums
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("q,tv_periodic,tv_open,s", [
    ([0, 5, 0], 10, 10, 5),
    ([1, 2, 3], 4, 2, 6),
    ([3, -2], 10, 5, 1),
    ([7], 0, 0, 7),
    ([4, 4, 4, 4], 0, 0, 16),
    ([2 ** 62, -(2 ** 62)], 2 ** 64, 2 ** 63, 0),
    ([2 ** 62 - 1] * 5, 0, 0, 5 * (2 ** 62 - 1)),
])
def test_invariants_hand_worked(q, tv_periodic, tv_open, s):
    a = O.invariants(np.array(q, dtype=np.int64), periodic=True)
    b = O.invariants(np.array(q, dtype=np.int64), periodic=False)
    assert a["tv"] == tv_periodic and b["tv"] == tv_open
    assert a["sum"] == s and b["sum"] == s
    assert a["min"] == min(q) and a["max"] == max(q)


def test_invariants_periodic_tv_is_rotation_invariant():
    q = W.random_states(101, -50, 50, seed=61)
    tv = O.invariants(q, periodic=True)["tv"]
    for k in (1, 17, 100):
        assert O.invariants(np.roll(q, k), periodic=True)["tv"] == tv


# ---------------------------------------------------------------------------
# Negative control (ii) of Thm transfer_operator_equivalence: the literal
# operation order of eq:flux_table, ((a*(delta*q))*lambda)/delta, is a
# different map from the canonical c*q on the first workload's state range,
# and it gives a different trajectory -- so the operation order is part of
# the method's definition at finite precision.
# ---------------------------------------------------------------------------
def test_literal_order_differs_from_canonical_upwind():
    w = W.w1_advection_square()
    p = O.Problem(O.UPWIND, w.delta, w.lam, width=32, a=1.0)
    q = np.arange(-20000, 20001, dtype=np.int64)
    literal = np.rint(((1.0 * (w.delta * q.astype(np.float64))) * w.lam) / w.delta).astype(np.int64)
    canonical = np.array([O.phi(p, True, int(v)) for v in q])
    differ = int(np.count_nonzero(literal != canonical))
    assert 500 < differ < 5000  # about 1.2k of 40001 states
    # and the trajectories part: step the first workload with the literal map
    q0 = O.quantise(w.u0, w.delta, 32)
    lit = q0.copy()
    for _ in range(200):
        phi = np.rint(((1.0 * (w.delta * lit.astype(np.float64))) * w.lam) / w.delta)
        phi = phi.astype(np.int64)
        lit = lit - (phi - np.roll(phi, 1))
    assert not np.array_equal(lit, O.step(p, q0, 200))


# ---------------------------------------------------------------------------
# The OpenMP build of the oracle gives the integers of the plain build.
# ---------------------------------------------------------------------------
def test_openmp_build_matches_plain_build():
    w = W.w2_burgers_step(n=1 << 14, steps=150)
    p = O.Problem(O.BURGERS_EO, w.delta, w.lam, width=32)
    q0 = O.quantise(w.u0, w.delta, 32)
    assert np.array_equal(O.step(p, q0, 150), O.step(p, q0, 150, omp=True))
    po = O.Problem(O.LF_BURGERS, 1e-3, 0.18, bc=O.OUTFLOW, alpha=2.5)
    qo = W.random_states(999, -800, 800, seed=67)
    a, la = O.step(po, qo, 40, return_ledger=True)
    b, lb = O.step(po, qo, 40, return_ledger=True, omp=True)
    assert np.array_equal(a, b) and la == lb
    w6 = W.w6_burgers_2d(nx=96, ny=64, steps=30)
    ax = [O.Problem(O.BURGERS_EO, w6.delta, w6.lam[0], width=32, bc=O.OUTFLOW),
          O.Problem(O.BURGERS_EO, w6.delta, w6.lam[1], width=32)]
    q6 = O.quantise(w6.u0, w6.delta, 32)
    a, la = O.step_nd(ax, q6, 30, return_ledger=True)
    b, lb = O.step_nd(ax, q6, 30, return_ledger=True, omp=True)
    assert np.array_equal(a, b) and la == lb
    r = W.sod_request(1500)
    pe = O.Problem(r.kind, r.delta, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
    q3 = np.stack([O.quantise(r.U0[c], r.delta) for c in range(3)])
    a, la = O.step_euler(pe, q3, 120, return_ledger=True)
    b, lb = O.step_euler(pe, q3, 120, return_ledger=True, omp=True)
    assert np.array_equal(a, b) and np.array_equal(la, lb)
