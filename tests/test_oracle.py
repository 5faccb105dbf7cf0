"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is a closed form, an
invariant the paper proves, an exact rational brute force, an exact solution,
or a hand-derived fixture under tests/golden/.  Runs without a GPU.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle import exact as X
from paper_2604_06947_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def read_golden(name):
    d = {}
    for line in open(__file__.rsplit("/", 1)[0] + "/golden/" + name):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        d[k] = v
    return d


# ---------------------------------------------------------------------------
# Quantisation (eq:quantisation) and reconstruction (eq:reconstruction_operator)
# ---------------------------------------------------------------------------
def test_quantise_rounds_half_to_even():
    d = 2.0 ** -10  # dyadic: u/delta is exact, so ties are real ties
    u = np.array([2.5, 3.5, -2.5, -0.5, 0.5, 1.5, 7.25, -7.75]) * d
    assert O.quantise(u, d).tolist() == [2, 4, -2, 0, 0, 2, 7, -8]


def test_reconstruct_is_delta_times_q():
    q = np.array([0, 1, -1, 123456789, -(2 ** 40)])
    assert np.array_equal(O.reconstruct(q, 0.25), q * 0.25)


def test_quantise_int32_range_error():
    with pytest.raises(O.OracleError):
        O.quantise(np.array([3.0e9]), 1.0, width=32)


# ---------------------------------------------------------------------------
# P1: upwind at c = 1/2 has an integer closed form for round-half-even(q/2)
# ---------------------------------------------------------------------------
def half_even_halves(q):
    return (q >> 1) + ((q & 1) & ((q >> 1) & 1))


def test_p1_upwind_half_closed_form_map():
    p = O.Problem(O.UPWIND, 1e-4, 0.5, a=1.0)
    for q in list(range(-50, 51)) + [-20001, -19999, 19999, 20001, 2 ** 31 - 1, -(2 ** 31)]:
        assert O.phi(p, True, q) == half_even_halves(q)
        assert O.phi(p, False, q) == 0


def test_p1_w1_trajectory_closed_form():
    w = W.w1_advection_square()
    q0 = O.quantise(w.u0, w.delta, 32)
    p = O.Problem(O.UPWIND, w.delta, w.lam, width=32, a=1.0)
    q = q0.copy()
    for _ in range(w.steps):  # q_i <- q_i - (g(q_i) - g(q_{i-1})), g = rint(q/2)
        g = half_even_halves(q)
        q = q - (g - np.roll(g, 1))
    assert np.array_equal(O.step(p, q0, w.steps), q)


# ---------------------------------------------------------------------------
# P2: upwind at c = +-1 is an exact one-cell shift per step
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("a", [1.0, -1.0])
def test_p2_unit_courant_shift(a):
    q0 = W.random_states(37, -1000, 1000, seed=7)
    p = O.Problem(O.UPWIND, 1e-3, 1.0, a=a)
    for s in (1, 5, 36):
        assert np.array_equal(O.step(p, q0, s), np.roll(q0, s if a > 0 else -s))
    assert np.array_equal(O.step(p, q0, 37), q0)


# ---------------------------------------------------------------------------
# P3: exact conservation (eq:exact_conservation); outflow ledger
# ---------------------------------------------------------------------------
KINDS = [
    (O.UPWIND, dict(a=1.0), 0.7),
    (O.UPWIND, dict(a=-0.8), 0.9),
    (O.BURGERS_EO, {}, None),
    (O.BURGERS_GODUNOV, {}, None),
    (O.BURGERS_MURMAN_ROE, {}, None),
    (O.LF_LINEAR, dict(a=0.6, alpha=1.0), 0.9),
    (O.LF_BURGERS, dict(alpha=2.0), None),
]


def burgers_problem(kind, u0, delta, bc, **kw):
    lam = 0.45 / float(np.max(np.abs(u0)))
    return O.Problem(kind, delta, lam, bc=bc, **kw)


@pytest.mark.parametrize("kind,kw,lam", KINDS)
@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW])
def test_p3_conservation_every_step(kind, kw, lam, bc):
    u0 = W.random_smooth_step(300, seed=11, b=0.2)
    delta = 1e-4
    if lam is None:
        lam = 0.45 / float(np.max(np.abs(u0)))
        if kind == O.LF_BURGERS:
            lam = 0.9 / kw["alpha"]
    p = O.Problem(kind, delta, lam, bc=bc, **kw)
    q = O.quantise(u0, delta)
    for _ in range(60):
        q1, led = O.step(p, q, 1, return_ledger=True)
        if bc == O.PERIODIC:
            assert led == 0
        assert int(q1.sum()) - int(q.sum()) == led
        q = q1


# ---------------------------------------------------------------------------
# P4: Lemma cfl_monotone (i)-(iii) and order preservation, for the kinds for
# which the rounded scheme is monotone; the LF counterexample is a fixture.
# ---------------------------------------------------------------------------
MONO = [
    (O.UPWIND, 0.3), (O.UPWIND, 0.5), (O.UPWIND, 0.9),
    (O.BURGERS_EO, 0.45), (O.BURGERS_EO, 0.95), (O.BURGERS_GODUNOV, 0.9),
]


@pytest.mark.parametrize("kind,cfl", MONO)
def test_p4_max_principle_tvd_l1_order(kind, cfl):
    n, delta = 257, 1e-4
    u0 = W.random_smooth_step(n, seed=21, b=0.1)
    v0 = u0 + W.random_smooth_step(n, seed=22, b=0.0) * 0.05
    v0 = np.maximum(v0, u0)  # ordered pair q0 <= p0
    if kind == O.UPWIND:
        p = O.Problem(kind, delta, cfl, a=1.0)
    else:
        lam = cfl / max(np.max(np.abs(u0)), np.max(np.abs(v0)))
        p = O.Problem(kind, delta, lam)
    q, r = O.quantise(u0, delta), O.quantise(v0, delta)
    lo, hi = q.min(), q.max()
    for _ in range(300):
        q1, r1 = O.step(p, q, 1), O.step(p, r, 1)
        assert q1.min() >= q.min() and q1.max() <= q.max()          # (i)
        assert O.invariants(q1)["tv"] <= O.invariants(q)["tv"]      # (ii)
        assert np.abs(q1 - r1).sum() <= np.abs(q - r).sum()         # (iii)
        assert np.all(q1 <= r1)                                     # order preservation
        q, r = q1, r1
    assert lo <= q.min() and q.max() <= hi


CERT = [(O.BURGERS_EO, 1e-5, 0.45, 1.0), (O.BURGERS_EO, 1e-5, 1.0, 1.0),
        (O.UPWIND, 1e-4, 0.9, 1.0), (O.UPWIND, 1e-4, 1.0, 1.0), (O.UPWIND, 1e-4, 0.9, -1.0),
        (O.UPWIND, 1e-4, 1.0, -1.0), (O.UPWIND, 1e-4, 0.5, 0.7)]


@pytest.mark.parametrize("kind,delta,cfl,a", CERT)
def test_p4_rounded_split_maps_certify_the_maximum_principle(kind, delta, cfl, a):
    """Lemma cfl_monotone on the rounded maps themselves: for CFL <= 1, from
    one state to the next phi+ rises by 0 or 1, phi- falls by 0 or 1, never
    both, so g(q) = q - phi+(q) + phi-(q) never falls.  Then the update
    g(q_i) + phi+(q_{i-1}) - phi-(q_{i+1}) is non-decreasing in each state and
    fixes constants, which is what lets the table path step without clamping.
    The regrouped form equals the oracle's step on random grids."""
    qmax = 30000
    if kind == O.UPWIND:
        p = O.Problem(kind, delta, cfl / abs(a), a=a)
    else:
        p = O.Problem(kind, delta, cfl / (delta * qmax))
    qs = np.arange(-qmax, qmax + 1)
    pp = np.array([O.phi(p, True, int(q)) for q in qs])
    pm = np.array([O.phi(p, False, int(q)) for q in qs])
    dp, dm = np.diff(pp), np.diff(pm)
    assert set(np.unique(dp)) <= {0, 1} and set(np.unique(dm)) <= {-1, 0}
    assert not np.any((dp != 0) & (dm != 0))
    g = qs - pp + pm
    assert np.all(np.diff(g) >= 0)
    rng = np.random.default_rng(5)
    for n in (3, 17, 256):
        q = rng.integers(-qmax, qmax + 1, n)
        i = q + qmax
        H = g[i] + pp[np.roll(i, 1)] - pm[np.roll(i, -1)]
        assert np.array_equal(O.step(p, q, 1), H)
        assert H.min() >= q.min() and H.max() <= q.max()


def test_p4_lf_counterexample_fixture():
    g = read_golden("lf_burgers_counterexample.txt")
    p = O.Problem(O.LF_BURGERS, float(g["delta"][0]), float(g["lambda"][0]),
                  alpha=float(g["alpha"][0]))
    q0 = np.array([int(v) for v in g["q0"]])
    q1 = np.array([int(v) for v in g["q1"]])
    assert O.phi(p, True, -496) == -101 and O.phi(p, False, -496) == 123
    assert O.phi(p, True, -495) == -100 and O.phi(p, False, -495) == 122
    out = O.step(p, q0, 1)
    assert np.array_equal(out, q1)
    assert out.min() < q0.min()  # the maximum principle fails for this kind


# ---------------------------------------------------------------------------
# P5: Prop. operator_quantisation_error with its sharp constant: each rounding
# contributes at most 1/2, so per step and cell the reconstructed increment
# differs from the classical split increment by at most 2 delta (split kinds,
# two roundings per interface) or delta (two-point kinds, one rounding).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,kw,bound", [
    (O.UPWIND, dict(a=1.0), 2), (O.UPWIND, dict(a=-1.0), 2), (O.BURGERS_EO, {}, 2),
    (O.LF_BURGERS, dict(alpha=1.8), 2), (O.LF_LINEAR, dict(a=0.5, alpha=1.0), 2),
    (O.BURGERS_GODUNOV, {}, 1), (O.BURGERS_MURMAN_ROE, {}, 1)])
def test_p5_sharp_per_step_bound(kind, kw, bound):
    n, delta = 400, 1e-5
    u0 = W.random_smooth_step(n, seed=31, b=0.3)
    lam = 0.4 / float(np.max(np.abs(u0)))
    if kind in (O.UPWIND,):
        lam = 0.73
    if kind in (O.LF_BURGERS, O.LF_LINEAR):
        lam = 0.5 / kw["alpha"]
    p = O.Problem(kind, delta, lam, **kw)
    q = O.quantise(u0, delta)
    worst = 0.0
    for _ in range(40):
        q1 = O.step(p, q, 1)
        u = O.reconstruct(q, delta)
        F = np.array([O.classical_flux(p, u[i], u[(i + 1) % n]) for i in range(n)])
        lamdF = lam * (F - np.roll(F, 1))
        res = np.abs(delta * (q1 - q).astype(np.float64) + lamdF)
        eps = 64 * 2.0 ** -53 * (np.abs(lam * F) + np.abs(lam * np.roll(F, 1)) + np.abs(u))
        assert np.all(res <= bound * delta + eps)
        worst = max(worst, float(np.max(res / delta)))
        q = q1
    assert worst > 0.25 * bound  # the bound is not vacuous on this data


# ---------------------------------------------------------------------------
# P6: Thm transfer_operator_equivalence / Remark godunov_lf_collapse.
# ---------------------------------------------------------------------------
def test_p6_equivalent_maps_identical_trajectories():
    n, delta = 512, 1e-5
    x = W.grid(n)
    u0 = 1.5 + np.sin(2 * np.pi * x) + 0.6 * (x >= 0.37)  # positive data
    lam = 0.45 / float(np.max(u0))
    q0 = O.quantise(u0, delta)
    traj = [O.step(O.Problem(k, delta, lam), q0, 600)
            for k in (O.BURGERS_EO, O.BURGERS_GODUNOV, O.BURGERS_MURMAN_ROE)]
    assert np.array_equal(traj[0], traj[1]) and np.array_equal(traj[0], traj[2])
    # the maps coincide on every visited interface state: positive states
    pe, pg = O.Problem(O.BURGERS_EO, delta, lam), O.Problem(O.BURGERS_GODUNOV, delta, lam)
    for qL, qR in [(5, 90000), (90000, 5), (123456, 123457)]:
        assert O.interface_flux(pe, qL, qR) == O.interface_flux(pg, qL, qR)


def test_p6_negative_control_mixed_sign():
    n, delta = 512, 1e-5
    u0 = 0.5 + np.sin(2 * np.pi * W.grid(n))  # Sec. 3.2 initial data: a shock with uL>0>uR forms
    lam = 0.45 / float(np.max(np.abs(u0)))
    q = O.quantise(u0, delta)
    pe, pg = O.Problem(O.BURGERS_EO, delta, lam), O.Problem(O.BURGERS_GODUNOV, delta, lam)
    a, b = q.copy(), q.copy()
    first = None
    for s in range(1, 1200):
        a, b = O.step(pe, a, 1), O.step(pg, b, 1)
        if not np.array_equal(a, b):
            first = s
            break
    assert first is not None and first > 50  # equal until a transonic shock forms
    # and on such a state pair the maps differ: EO adds f-(uR) > 0
    assert O.interface_flux(pe, 50000, -40000) != O.interface_flux(pg, 50000, -40000)


# ---------------------------------------------------------------------------
# P7: a constant state is a fixed point of every kind
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,kw", [(O.UPWIND, dict(a=0.9)), (O.UPWIND, dict(a=-0.4)),
                                     (O.BURGERS_EO, {}), (O.BURGERS_GODUNOV, {}),
                                     (O.LF_LINEAR, dict(a=0.5, alpha=1.0)),
                                     (O.LF_BURGERS, dict(alpha=2.0)),
                                     (O.BURGERS_MURMAN_ROE, {})])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW])
def test_p7_constant_state_fixed_point(kind, kw, bc):
    p = O.Problem(kind, 1e-4, 0.3, bc=bc, **kw)
    for c in (-7777, 0, 12345):
        q = np.full(33, c)
        assert np.array_equal(O.step(p, q, 25), q)


@pytest.mark.parametrize("kind", [O.EULER_ROE, O.EULER_ROE_EF])
def test_p7_euler_constant_state_fixed_point(kind):
    p = O.Problem(kind, 1e-6, 0.3, bc=O.OUTFLOW)
    U = np.stack([np.full(20, 0.7), np.full(20, 0.3), np.full(20, 2.1)])
    q = np.stack([O.quantise(U[c], 1e-6) for c in range(3)])
    assert np.array_equal(O.step_euler(p, q, 30), q)


# ---------------------------------------------------------------------------
# P8: exhaustive brute force on tiny grids against exact rational arithmetic.
# With dyadic delta, dt/dx, a and alpha every canonical FP64 expression is
# exact, so the oracle must equal round-half-even of the exact rationals.
# ---------------------------------------------------------------------------
def frac_maps(kind, delta, lam, a, alpha):
    d, L, A, al = Fraction(delta), Fraction(lam), Fraction(a), Fraction(alpha)

    def f(u):
        return A * u if kind == O.LF_LINEAR else u * u / 2

    def phi_p(q):
        u = d * q
        if kind == O.UPWIND:
            return round(max(A, 0) * u * L / d)
        if kind == O.BURGERS_EO:
            return round(max(u, 0) ** 2 / 2 * L / d)
        return round((f(u) + al * u) / 2 * L / d)

    def phi_m(q):
        u = d * q
        if kind == O.UPWIND:
            return round(min(A, 0) * u * L / d)
        if kind == O.BURGERS_EO:
            return round(min(u, 0) ** 2 / 2 * L / d)
        return round((f(u) - al * u) / 2 * L / d)

    def flux(qL, qR):
        if kind in (O.BURGERS_GODUNOV, O.BURGERS_MURMAN_ROE):
            uL, uR = d * qL, d * qR
            if kind == O.BURGERS_MURMAN_ROE:
                fl = uL * uL / 2 if uL + uR >= 0 else uR * uR / 2
            elif uL <= uR:  # min of f over [uL, uR]
                fl = 0 if uL <= 0 <= uR else min(uL * uL, uR * uR) / 2
            else:           # max of f over [uR, uL]
                fl = max(uL * uL, uR * uR) / 2
            return round(fl * L / d)
        return phi_p(qL) + phi_m(qR)

    return flux


def frac_step(flux, q, bc):
    n = len(q)
    if bc == O.PERIODIC:
        F = [flux(q[i - 1], q[i]) for i in range(n)] + [flux(q[n - 1], q[0])]
    else:
        F = [flux(q[0], q[0])] + [flux(q[i - 1], q[i]) for i in range(1, n)] + \
            [flux(q[n - 1], q[n - 1])]
    return [q[i] - (F[i + 1] - F[i]) for i in range(n)]


BRUTE = [
    (O.UPWIND, 0.5, 1.0, 0.0), (O.UPWIND, 0.75, -1.0, 0.0), (O.UPWIND, 0.75, 0.75, 0.0),
    (O.BURGERS_EO, 0.5, 1.0, 0.0), (O.BURGERS_EO, 0.25, 1.0, 0.0),
    (O.BURGERS_GODUNOV, 0.5, 1.0, 0.0), (O.BURGERS_MURMAN_ROE, 0.75, 1.0, 0.0),
    (O.LF_LINEAR, 0.25, 0.5, 1.0), (O.LF_BURGERS, 0.25, 1.0, 2.0),
]


@pytest.mark.parametrize("kind,lam,a,alpha", BRUTE)
@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW])
def test_p8_exhaustive_tiny_grids(kind, lam, a, alpha, bc):
    import itertools
    delta = 0.5
    flux = frac_maps(kind, delta, lam, a, alpha)
    p = O.Problem(kind, delta, lam, bc=bc, a=a, alpha=alpha)
    cases = []
    for n in (1, 2, 3):
        cases += [list(t) for t in itertools.product(range(-4, 5), repeat=n)]
    rng = np.random.default_rng(8)
    cases += [list(rng.integers(-4, 5, size=n)) for n in (4, 5) for _ in range(150)]
    for q0 in cases:
        ref = [int(v) for v in q0]
        got = np.array(q0, dtype=np.int64)
        for _ in range(8):
            ref = frac_step(flux, ref, bc)
            got = O.step(p, got, 1)
            assert got.tolist() == ref, (q0, kind)


# ---------------------------------------------------------------------------
# P9: symmetries
# ---------------------------------------------------------------------------
def test_p9_eo_mirror_symmetry():
    n, delta = 301, 1e-5
    u0 = 0.5 + np.sin(2 * np.pi * W.grid(n)) + 0.4 * (W.grid(n) > 0.6)
    lam = 0.45 / float(np.max(np.abs(u0)))
    p = O.Problem(O.BURGERS_EO, delta, lam)
    q = O.quantise(u0, delta)
    qm = -q[::-1]
    for _ in range(5):
        q, qm = O.step(p, q, 80), O.step(p, qm, 80)
        assert np.array_equal(qm, -q[::-1])


@pytest.mark.parametrize("kind", [O.UPWIND, O.BURGERS_EO, O.BURGERS_GODUNOV])
def test_p9_translation_commutes(kind):
    n, delta = 200, 1e-5
    u0 = W.random_smooth_step(n, seed=41)
    lam = 0.45 / float(np.max(np.abs(u0)))
    p = O.Problem(kind, delta, lam, a=1.0)
    q = O.quantise(u0, delta)
    for s in (1, 17, 199):
        assert np.array_equal(O.step(p, np.roll(q, s), 90), np.roll(O.step(p, q, 90), s))


def test_p9_single_cell_periodic_never_changes():
    for kind in (O.UPWIND, O.BURGERS_EO, O.LF_BURGERS, O.BURGERS_GODUNOV):
        p = O.Problem(kind, 1e-3, 0.4, alpha=2.0)
        assert O.step(p, np.array([4321]), 50).tolist() == [4321]


# ---------------------------------------------------------------------------
# P10: exact references (Thm convergence; Sec. 3 experiments)
# ---------------------------------------------------------------------------
def test_p10_advection_unit_courant_matches_exact_shift():
    n = 256
    w = W.w1_advection_square(n=n)
    p = O.Problem(O.UPWIND, w.delta, 1.0, a=1.0)
    q = O.step(p, O.quantise(w.u0, w.delta), 64)  # t = 64 dx = 0.25
    ref = X.shift(lambda x: ((x >= 0.25) & (x <= 0.5)) + 0.3 * np.sin(2 * np.pi * x),
                  W.grid(n), 0.25)
    assert np.max(np.abs(O.reconstruct(q, w.delta) - ref)) <= 0.5 * w.delta + 1e-12


def test_p10_burgers_converges_to_hopf_lax():
    data = X.SineStepData(b=0.5, A=1.0)  # Sec. 3.2: u0 = 0.5 + sin(2 pi x)
    t = 0.3  # past the shock formation time 1/(2 pi)
    errs = []
    for n in (128, 256, 512):
        u0 = data.u0(W.grid(n))
        delta = 1e-3 / n  # delta/dx -> 0
        lam = 0.45 / float(np.max(np.abs(u0)))
        steps = int(round(t / (lam / n)))
        lam = t / (steps / n)
        p = O.Problem(O.BURGERS_EO, delta, lam)
        u = O.reconstruct(O.step(p, O.quantise(u0, delta), steps), delta)
        ref = X.hopf_lax_burgers(data, W.grid(n), t)
        errs.append(float(np.mean(np.abs(u - ref))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.02


def test_p10_sod_exact_reference_and_fixture():
    g = read_golden("sod_exact_star.txt")
    ps, us = X.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert abs(ps - float(g["p_star"][0])) < 1e-5 and abs(us - float(g["u_star"][0])) < 1e-5
    S = X.shock_speed_right((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert abs(S - float(g["shock_speed"][0])) < 1e-5
    assert abs(0.5 + 0.2 * S - float(g["shock_x_at_t0.2"][0])) < 1e-5
    rho, _, _ = X.riemann_exact((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), np.array([0.5, 1.0]))
    assert abs(rho[0] - float(g["rho_star_left"][0])) < 1e-5
    assert abs(rho[1] - float(g["rho_star_right"][0])) < 1e-5


@pytest.mark.parametrize("kind", [O.EULER_ROE_EF, O.EULER_ROE])
def test_p10_quantised_sod_against_exact(kind):
    n = 1024
    r = W.sod_request(n, kind=kind)
    p = O.Problem(kind, r.delta, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
    q0 = np.stack([O.quantise(r.U0[c], r.delta) for c in range(3)])
    q = O.step_euler(p, q0, r.steps)
    rho = O.reconstruct(q[0], r.delta)
    x = W.grid(n)
    xd = (n // 2 - 0.5) / n
    ref, _, _ = X.riemann_exact(r.left, r.right, (x - xd) / r.t_final)
    err = float(np.mean(np.abs(rho - ref)))
    fp = O.classical_step_euler(p, O.reconstruct(q0.ravel(), r.delta).reshape(3, n), r.steps)
    err_fp = float(np.mean(np.abs(fp[0] - ref)))
    assert err <= 0.02 and err <= 2 * err_fp
    # shock position: the density midpoint between star-right and right states
    mid = 0.5 * (0.26557 + 0.125)
    k = np.where((rho[:-1] > mid) & (rho[1:] <= mid))[0]
    xs = x[k[-1]]
    assert abs(xs - 0.8504) < 4.0 / n


# ---------------------------------------------------------------------------
# P11: checkpoint / resume is exact (the integer state is the full state)
# ---------------------------------------------------------------------------
def test_p11_checkpoint_resume():
    w = W.w2_burgers_step(n=4096, steps=300)
    p = O.Problem(O.BURGERS_EO, w.delta, w.lam, width=32)
    q0 = O.quantise(w.u0, w.delta, 32)
    a = O.step(p, q0, 300)
    b = O.step(p, O.step(p, q0, 113), 187)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Euler: the Roe linearisation (Sec. 3.3 uses a Roe-type flux).  Pinned by the
# defining properties of the Roe matrix: sum a_k r_k = dU and
# sum l_k a_k r_k = f(U_R) - f(U_L), independent of the flux formula.
# ---------------------------------------------------------------------------
def test_euler_roe_linearisation_properties():
    delta = 1e-6
    p = O.Problem(O.EULER_ROE, delta, 0.3, gamma=1.4)
    rng = np.random.default_rng(12)
    for _ in range(50):
        r = rng.uniform(0.1, 2.0, 2)
        u = rng.uniform(-1.0, 1.0, 2)
        pr = rng.uniform(0.1, 2.0, 2)
        U = np.array([r, r * u, pr / 0.4 + 0.5 * r * u * u])
        qL, qR = O.quantise(U[:, 0], delta), O.quantise(U[:, 1], delta)
        F, wv = O.euler_flux(p, qL, qR)
        ub, Hb, cb, c2, a1, a2, a3, l1, l2, l3 = wv
        R = np.array([[1, ub - cb, Hb - ub * cb], [1, ub, 0.5 * ub * ub],
                      [1, ub + cb, Hb + ub * cb]])
        A = np.array([a1, a2, a3])
        L = np.array([l1, l2, l3])
        ULr, URr = delta * qL.astype(float), delta * qR.astype(float)

        def phys(Uc):
            rr, mm, EE = Uc
            uu = mm / rr
            pp = 0.4 * (EE - 0.5 * mm * uu)
            return np.array([mm, mm * uu + pp, uu * (EE + pp)])

        dU = URr - ULr
        dF = phys(URr) - phys(ULr)
        assert np.allclose(A @ R, dU, rtol=1e-9, atol=1e-9)
        assert np.allclose((A * L) @ R, dF, rtol=1e-9, atol=1e-9)
        # and the flux itself: F = (fL + fR)/2 - 1/2 sum |l_k| a_k r_k
        Fref = 0.5 * (phys(ULr) + phys(URr)) - 0.5 * (np.abs(L) * A) @ R
        assert np.allclose(F, Fref, rtol=1e-12, atol=1e-12)


def test_euler_supersonic_interface_is_upwind():
    delta = 1e-6
    for kind in (O.EULER_ROE, O.EULER_ROE_EF):
        p = O.Problem(kind, delta, 0.3, gamma=1.4)
        U = lambda r, u, pr: np.array([r, r * u, pr / 0.4 + 0.5 * r * u * u])
        qL = O.quantise(U(1.0, 3.0, 1.0), delta)
        qR = O.quantise(U(0.9, 3.1, 0.9), delta)
        F, wv = O.euler_flux(p, qL, qR)
        assert wv[7] > 0  # all waves move right
        uL = delta * qL.astype(float)
        uu = uL[1] / uL[0]
        pp = 0.4 * (uL[2] - 0.5 * uL[1] * uu)
        assert np.allclose(F, [uL[1], uL[1] * uu + pp, uu * (uL[2] + pp)], rtol=1e-12)


def test_euler_conservation_with_outflow_ledger():
    r = W.sod_request(256)
    p = O.Problem(r.kind, r.delta, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
    q = np.stack([O.quantise(r.U0[c], r.delta) for c in range(3)])
    for _ in range(20):
        q1, led = O.step_euler(p, q, 7, return_ledger=True)
        assert np.array_equal(q1.sum(axis=1) - q.sum(axis=1), led)
        q = q1


# ---------------------------------------------------------------------------
# Level statistics (Supplementary Information)
# ---------------------------------------------------------------------------
def test_entropy_log_count():
    q = np.repeat(np.arange(-3, 4), 5)  # uniform on 7 levels
    assert abs(O.entropy(q) - math.log(7)) < 1e-14
    assert O.entropy(np.full(10, 3)) == 0.0


def test_level_transition_counts_are_consistent():
    w = W.w2_burgers_step(n=2048, steps=1)
    p = O.Problem(O.BURGERS_EO, 1e-3, w.lam)
    q0 = O.quantise(w.u0, 1e-3)
    q1 = O.step(p, q0, 400)
    q2 = O.step(p, q1, 1)
    f, t, c = O.level_transitions(q1, q2)
    lv1, c1 = O.level_histogram(q1)
    lv2, c2 = O.level_histogram(q2)
    # column sums give c^n, row sums give c^{n+1} (Definition level_transition)
    for k, ck in zip(lv1, c1):
        assert c[f == k].sum() == ck
    for k, ck in zip(lv2, c2):
        assert c[t == k].sum() == ck
    assert c.sum() == q1.size


def test_row_defect_hand_examples():
    # [0,0,1] -> [1,0,0]: N_00 = N_10 = N_01 = 1, c_0 = 2, c_1 = 1, so
    # row 0 sums to 1/2 + 1 and row 1 to 1/2: rho = 1/2 (worked by hand)
    assert O.row_defect([0, 0, 1], [1, 0, 0]) == 0.5
    # [0,1] -> [1,1]: level 0 empties, row 1 = 1/1 + 1/1 = 2
    assert O.row_defect([0, 1], [1, 1]) == 1.0
    # identity, a shift of every level, and an even mixing of two equal levels
    # are doubly stochastic
    q = np.array([3, -1, 3, 0, 0, 0, 7])
    assert O.row_defect(q, q) == 0.0
    assert O.row_defect(q, q + 7) == 0.0
    assert O.row_defect([0, 0, 1, 1], [0, 1, 0, 1]) == 0.0
    assert O.row_defect([], []) == 0.0


def _dense_transition_matrix(q0, q1):
    """Brute force: M as a dense matrix over the union of levels, one cell at a time."""
    lv = sorted(set(int(x) for x in q0) | set(int(x) for x in q1))
    ix = {k: j for j, k in enumerate(lv)}
    N = np.zeros((len(lv), len(lv)))
    for a, b in zip(q0, q1):
        N[ix[int(b)], ix[int(a)]] += 1
    c0 = np.array([sum(1 for a in q0 if a == k) for k in lv], dtype=float)
    M = np.divide(N, c0[None, :], out=np.zeros_like(N), where=c0[None, :] > 0)
    return lv, M, c0


@pytest.mark.parametrize("seed", range(6))
def test_row_defect_matches_dense_matrix(seed):
    rng = np.random.default_rng(seed)
    n = 40
    q0 = rng.integers(-3, 4, n)
    q1 = q0 + rng.integers(-1, 2, n)
    lv, M, c0 = _dense_transition_matrix(q0, q1)
    p0 = c0 / n
    p1 = np.array([sum(1 for b in q1 if b == k) for k in lv], dtype=float) / n
    # eq:pn1_equals_Mpn and column-stochasticity on the occupied levels
    assert np.allclose(M @ p0, p1, atol=1e-15)
    assert np.allclose(M.sum(axis=0)[c0 > 0], 1.0, atol=1e-15)
    rows = M.sum(axis=1)[p1 > 0]
    assert abs(O.row_defect(q0, q1) - np.abs(rows - 1.0).max()) < 1e-14
    # the entries of M add up to the number of levels occupied before the step
    assert abs(rows.sum() - np.count_nonzero(c0)) < 1e-12


def test_row_defect_zero_implies_entropy_does_not_drop():
    # equal level counts permuted among cells: M is doubly stochastic
    # (Remark doubly_stochastic_condition) and the entropy cannot decrease
    # (Theorem entropy_increase); here it is unchanged
    rng = np.random.default_rng(5)
    q0 = np.repeat(np.arange(-5, 6), 9)
    q1 = rng.permutation(q0)
    # each row is a sum of ninths that add up to one, up to rounding
    assert O.row_defect(q0, q1) < 4e-16
    assert O.entropy(q1) >= O.entropy(q0) - 1e-15


# Transonic rarefactions (left-going, and its mirror image right-going): plain
# Roe admits an entropy-violating expansion jump at the sonic point, and the
# entropy fix of the acoustic waves removes it, so against the exact solution
# the fixed flux must be clearly closer.  The two cases exercise the fix of
# the 1-wave and of the 3-wave respectively.
@pytest.mark.parametrize("left,right", [((1.0, 0.75, 1.0), (0.125, 0.0, 0.1)),
                                        ((0.125, 0.0, 0.1), (1.0, -0.75, 1.0))])
def test_p10_transonic_rarefaction_entropy_fix(left, right):
    n = 512
    errs = {}
    for kind in (O.EULER_ROE, O.EULER_ROE_EF):
        r = W.sod_request(n, left, right, kind=kind)
        p = O.Problem(kind, r.delta, r.lam, bc=O.OUTFLOW, gamma=1.4)
        q0 = np.stack([O.quantise(r.U0[c], r.delta) for c in range(3)])
        rho = O.reconstruct(O.step_euler(p, q0, r.steps)[0], r.delta)
        x = W.grid(n)
        ref, _, _ = X.riemann_exact(left, right, (x - (n // 2 - 0.5) / n) / r.t_final)
        errs[kind] = float(np.mean(np.abs(rho - ref)))
    assert errs[O.EULER_ROE_EF] < 0.8 * errs[O.EULER_ROE]
    assert errs[O.EULER_ROE_EF] < 0.008


@pytest.mark.parametrize("kind", [O.EULER_ROE, O.EULER_ROE_EF])
def test_euler_mirror_symmetry(kind):
    """Reflection x -> -x (rho, E even; m odd) maps solutions to solutions.  A
    fix applied differently to the 1- and 3-waves breaks it.  Summation order
    can differ between an interface and its mirror, so up to 2 counts of
    difference are allowed; the runs seen so far agree bitwise."""
    n = 512

    def run(left, right):
        r = W.sod_request(n, left, right, kind=kind)
        p = O.Problem(kind, r.delta, r.lam, bc=O.OUTFLOW, gamma=1.4)
        q0 = np.stack([O.quantise(r.U0[c], r.delta) for c in range(3)])
        return O.step_euler(p, q0, r.steps)

    a = run((1.0, 0.75, 1.0), (0.125, 0.0, 0.1))
    b = run((0.125, 0.0, 0.1), (1.0, -0.75, 1.0))
    assert np.abs(a[0] - b[0][::-1]).max() <= 2
    assert np.abs(a[1] + b[1][::-1]).max() <= 2
    assert np.abs(a[2] - b[2][::-1]).max() <= 2


# ---------------------------------------------------------------------------
# Density-only quantisation of the Roe update (Sec. 3.3, the prototype the
# paper runs): integer density, real momentum and energy.
# ---------------------------------------------------------------------------
def _sod_density_state(r):
    return O.quantise(r.U0[0], r.delta), r.U0[1].copy(), r.U0[2].copy()


@pytest.mark.parametrize("kind", [O.EULER_ROE, O.EULER_ROE_EF])
def test_density_only_one_step_against_fp64_roe(kind):
    # From the same state the fluxes are the FP64 scheme's own, so after one
    # step m and E equal the classical update bit for bit, and the density
    # differs from it only by the two roundings of its transfers: at most delta
    # (each transfer within delta/2 of lambda*F_rho).
    rng = np.random.default_rng(41)
    n = 300
    r = W.sod_request(n, kind=kind)
    p = O.Problem(kind, r.delta, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
    qr = O.quantise(r.U0[0] * (1 + 0.1 * rng.random(n)), r.delta)
    m = r.U0[1] + 0.05 * rng.standard_normal(n)  # keeps the pressure positive
    E = r.U0[2] * (1 + 0.1 * rng.random(n))
    q1, m1, E1 = O.step_euler_density(p, qr, m, E, 1)
    U = np.stack([O.reconstruct(qr, r.delta), m, E])
    fp = O.classical_step_euler(p, U, 1)
    assert np.array_equal(m1.view(np.uint64), fp[1].view(np.uint64))
    assert np.array_equal(E1.view(np.uint64), fp[2].view(np.uint64))
    assert np.abs(O.reconstruct(q1, r.delta) - fp[0]).max() <= r.delta * (1 + 1e-9)


def test_density_only_conservation_and_fixed_point():
    r = W.sod_request(400)
    p = O.Problem(O.EULER_ROE_EF, r.delta, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
    qr, m, E = _sod_density_state(r)
    cur, led_total = qr, 0
    mm, EE = m, E
    for _ in range(30):
        nxt, mm, EE, led = O.step_euler_density(p, cur, mm, EE, 1, return_ledger=True)
        assert int(nxt.sum()) - int(cur.sum()) == led
        led_total += led
        cur = nxt
    pp = O.Problem(O.EULER_ROE_EF, r.delta, r.lam, bc=O.PERIODIC, gamma=r.gamma)
    a, _, _ = O.step_euler_density(pp, qr, m, E, 50)
    assert int(a.sum()) == int(qr.sum())
    const = O.step_euler_density(p, np.full(20, 700000), np.full(20, 0.2), np.full(20, 2.5), 40)
    assert np.all(const[0] == 700000) and np.all(const[1] == 0.2) and np.all(const[2] == 2.5)


@pytest.mark.parametrize("kind", [O.EULER_ROE_EF, O.EULER_ROE])
def test_density_only_sod_against_exact(kind):
    # the paper's experiment: Sod at t = 0.2 against the exact Riemann solution
    n = 1024
    r = W.sod_request(n, kind=kind)
    p = O.Problem(kind, r.delta, r.lam, bc=O.OUTFLOW, gamma=r.gamma)
    qr, m, E = _sod_density_state(r)
    q, m1, E1 = O.step_euler_density(p, qr, m, E, r.steps)
    rho = O.reconstruct(q, r.delta)
    x = W.grid(n)
    xd = (n // 2 - 0.5) / n
    ref, _, _ = X.riemann_exact(r.left, r.right, (x - xd) / r.t_final)
    err = float(np.mean(np.abs(rho - ref)))
    fp = O.classical_step_euler(p, np.stack([O.reconstruct(qr, r.delta), m, E]), r.steps)
    err_fp = float(np.mean(np.abs(fp[0] - ref)))
    assert err <= 0.02 and err <= 2 * err_fp
    mid = 0.5 * (0.26557 + 0.125)
    k = np.where((rho[:-1] > mid) & (rho[1:] <= mid))[0]
    assert abs(x[k[-1]] - 0.8504) < 4.0 / n


def test_density_only_mirror_symmetry():
    n = 512

    def run(left, right):
        r = W.sod_request(n, left, right, kind=O.EULER_ROE_EF)
        p = O.Problem(O.EULER_ROE_EF, r.delta, r.lam, bc=O.OUTFLOW, gamma=1.4)
        return O.step_euler_density(p, *_sod_density_state(r), r.steps)

    a = run((1.0, 0.75, 1.0), (0.125, 0.0, 0.1))
    b = run((0.125, 0.0, 0.1), (1.0, -0.75, 1.0))
    assert np.abs(a[0] - b[0][::-1]).max() <= 2
    assert np.abs(a[1] + b[1][::-1]).max() <= 1e-9
    assert np.abs(a[2] - b[2][::-1]).max() <= 1e-9
