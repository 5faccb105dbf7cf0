"""Pins of the oracle's d-dimensional directional composition
(Thm dimension_extension, eq:nd_transfer_rule, eq:nd_flux_definition).

What fixes it independently of its own code: an exact-rational brute force on
tiny 2-D and 3-D grids, reductions to the (separately pinned) one-dimensional
update, exact shifts, conservation and the boundary ledger, the monotone-scheme
properties under a summed CFL number <= 1, and the symmetries of the Cartesian
grid (axis permutation, translation)."""
import itertools

import numpy as np
import pytest

import oracle as O
from test_oracle import frac_maps


def P(kind, lam, bc=O.PERIODIC, a=1.0, alpha=0.0, delta=0.5, width=64):
    return O.Problem(kind, delta, lam, bc=bc, width=width, a=a, alpha=alpha)


def frac_step_nd(fluxes, bcs, q):
    """One step of eq:nd_transfer_rule on a nested-list grid, exact rationals.
    q is indexed q[i_{d-1}]...[i_0]; fluxes[m], bcs[m] belong to axis m (i_m)."""
    a = np.array(q, dtype=object)
    d = a.ndim
    out = a.copy()
    for idx in itertools.product(*[range(s) for s in a.shape]):
        c = a[idx]  # every flux from the state before the step
        v = c
        for m in range(d):
            ax = d - 1 - m  # numpy axis of direction m
            n = a.shape[ax]
            i = idx[ax]

            def nb(j):
                t = list(idx)
                t[ax] = j
                return a[tuple(t)]
            if i + 1 < n:
                right = nb(i + 1)
            else:
                right = nb(0) if bcs[m] == O.PERIODIC else c
            if i > 0:
                left = nb(i - 1)
            else:
                left = nb(n - 1) if bcs[m] == O.PERIODIC else c
            v = v - (fluxes[m](c, right) - fluxes[m](left, c))
        out[idx] = v
    return out


CASES_2D = [
    # kind, (lam_x, a_x, alpha_x), (lam_y, a_y, alpha_y)
    (O.UPWIND, (0.5, 1.0, 0.0), (0.25, -1.0, 0.0)),
    (O.UPWIND, (0.25, 0.75, 0.0), (0.5, 1.0, 0.0)),
    (O.BURGERS_EO, (0.25, 1.0, 0.0), (0.125, 1.0, 0.0)),
    (O.BURGERS_GODUNOV, (0.25, 1.0, 0.0), (0.25, 1.0, 0.0)),
    (O.BURGERS_MURMAN_ROE, (0.125, 1.0, 0.0), (0.25, 1.0, 0.0)),
    (O.LF_LINEAR, (0.25, 0.5, 1.0), (0.125, -0.5, 1.0)),
    (O.LF_BURGERS, (0.125, 1.0, 2.0), (0.125, 1.0, 2.0)),
]


@pytest.mark.parametrize("kind,px,py", CASES_2D)
@pytest.mark.parametrize("bcx,bcy", [(O.PERIODIC, O.PERIODIC), (O.OUTFLOW, O.OUTFLOW),
                                     (O.PERIODIC, O.OUTFLOW)])
def test_nd_brute_force_2d(kind, px, py, bcx, bcy):
    delta = 0.5
    fx = frac_maps(kind, delta, px[0], px[1], px[2])
    fy = frac_maps(kind, delta, py[0], py[1], py[2])
    ax = [P(kind, px[0], bcx, a=px[1], alpha=px[2]), P(kind, py[0], bcy, a=py[1], alpha=py[2])]
    rng = np.random.default_rng(20)
    shapes = [(1, 1), (1, 3), (3, 1), (2, 2), (2, 3), (3, 2), (3, 4)]
    for shp in shapes:
        for _ in range(25):
            q0 = rng.integers(-4, 5, size=shp)
            ref = q0.astype(object)
            got = q0.copy()
            for _ in range(5):
                ref = frac_step_nd([fx, fy], [bcx, bcy], ref)
                got = O.step_nd(ax, got, 1)
                assert got.tolist() == ref.tolist(), (shp, q0.tolist())


@pytest.mark.parametrize("kind", [O.UPWIND, O.BURGERS_EO, O.BURGERS_GODUNOV])
def test_nd_brute_force_3d(kind):
    delta = 0.5
    lams = (0.25, 0.125, 0.125)
    a_s = (1.0, -1.0, 0.5)
    fl = [frac_maps(kind, delta, lams[m], a_s[m], 0.0) for m in range(3)]
    bcs = [O.PERIODIC, O.OUTFLOW, O.PERIODIC]
    ax = [P(kind, lams[m], bcs[m], a=a_s[m]) for m in range(3)]
    rng = np.random.default_rng(21)
    for shp in [(2, 2, 2), (1, 2, 3), (3, 2, 1), (2, 3, 2)]:
        for _ in range(10):
            q0 = rng.integers(-4, 5, size=shp)
            ref = q0.astype(object)
            got = q0.copy()
            for _ in range(4):
                ref = frac_step_nd(fl, bcs, ref)
                got = O.step_nd(ax, got, 1)
                assert got.tolist() == ref.tolist(), (shp, q0.tolist())


@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW])
def test_nd_reduces_to_1d(bc):
    # a single row (or column) is the one-dimensional update of its axis; data
    # constant along x evolves as the one-dimensional update along y
    rng = np.random.default_rng(3)
    px = P(O.BURGERS_EO, 0.2, bc, delta=1e-3)
    py = P(O.BURGERS_EO, 0.15, bc, delta=1e-3)
    row = rng.integers(-700, 900, size=57)
    assert np.array_equal(O.step_nd([px, py], row[None, :], 30)[0], O.step(px, row, 30))
    assert np.array_equal(O.step_nd([px, py], row[:, None], 30)[:, 0], O.step(py, row, 30))
    grid = np.repeat(row[:, None], 13, axis=1)  # q[j, i] = row[j]
    got = O.step_nd([px, py], grid, 30)
    ref = O.step(py, row, 30)
    assert np.array_equal(got, np.repeat(ref[:, None], 13, axis=1))


def test_nd_exact_shifts():
    # UPWIND with c_x = 1, c_y = 0 shifts every row by one cell; c_y = -1 shifts columns
    rng = np.random.default_rng(4)
    q = rng.integers(-10 ** 6, 10 ** 6, size=(9, 11))
    sx = O.step_nd([P(O.UPWIND, 1.0, a=1.0, delta=1e-3), P(O.UPWIND, 1.0, a=0.0, delta=1e-3)],
                   q, 1)
    assert np.array_equal(sx, np.roll(q, 1, axis=1))
    sy = O.step_nd([P(O.UPWIND, 1.0, a=0.0, delta=1e-3), P(O.UPWIND, 1.0, a=-1.0, delta=1e-3)],
                   q, 1)
    assert np.array_equal(sy, np.roll(q, -1, axis=0))
    q3 = rng.integers(-1000, 1000, size=(4, 5, 6))
    s3 = O.step_nd([P(O.UPWIND, 1.0, a=0.0, delta=1e-3), P(O.UPWIND, 1.0, a=0.0, delta=1e-3),
                    P(O.UPWIND, 1.0, a=1.0, delta=1e-3)], q3, 1)
    assert np.array_equal(s3, np.roll(q3, 1, axis=0))


def test_nd_conservation_and_ledger():
    rng = np.random.default_rng(5)
    q = rng.integers(-3000, 5000, size=(24, 31))
    ax = [P(O.BURGERS_GODUNOV, 0.06, delta=1e-3), P(O.BURGERS_GODUNOV, 0.05, delta=1e-3)]
    assert O.step_nd(ax, q, 40).sum() == q.sum()
    ax = [P(O.BURGERS_EO, 0.06, O.OUTFLOW, delta=1e-3), P(O.BURGERS_EO, 0.05, O.OUTFLOW, delta=1e-3)]
    led_total = 0
    cur = q.copy()
    for _ in range(40):
        nxt, led = O.step_nd(ax, cur, 1, return_ledger=True)
        # the step's mass change is exactly the boundary ledger of that step
        assert nxt.sum() - cur.sum() == led
        led_total += led
        cur = nxt
    q40, led40 = O.step_nd(ax, q, 40, return_ledger=True)
    assert np.array_equal(q40, cur) and led40 == led_total
    assert led_total != 0


def test_nd_max_principle_fails_by_one_count():
    # Thm dimension_extension promises conservation, linear cost and O(delta)
    # consistency, not monotonicity, and the composed quantised update is not
    # monotone: with split maps the rounding steps of two directions can add up.
    # Worked by hand: UPWIND, c_x = c_y = 1/2 (summed CFL 1), phi(q) = rint(q/2).
    # A cell holding 3 with zero neighbours sends rint(3/2) = 2 counts across
    # each of its two outflow faces and keeps 3 - 4 = -1, below the initial
    # minimum 0; the cell holding 1 keeps 1 - 0 - 0 = 1, so the order of the two
    # states (3 > 1) flips.
    ax = [P(O.UPWIND, 0.5, a=1.0, delta=1e-3), P(O.UPWIND, 0.5, a=1.0, delta=1e-3)]
    q3 = np.zeros((4, 4), dtype=np.int64)
    q3[1, 1] = 3
    q1 = np.zeros((4, 4), dtype=np.int64)
    q1[1, 1] = 1
    a, b = O.step_nd(ax, q3, 1), O.step_nd(ax, q1, 1)
    assert a[1, 1] == -1 and a.min() == -1
    assert b[1, 1] == 1
    assert a.sum() == 3 and b.sum() == 1  # still conservative
    # in one dimension the same maps keep the maximum principle (P4): 3 -> 3 - 2 = 1
    assert O.step(P(O.UPWIND, 0.5, a=1.0, delta=1e-3), np.array([0, 3, 0, 0]), 1).min() == 0


def test_nd_axis_permutation_and_translation():
    rng = np.random.default_rng(7)
    q = rng.integers(-2000, 2000, size=(10, 14))
    px = P(O.LF_BURGERS, 0.2, alpha=2.0, delta=1e-3)
    py = P(O.LF_BURGERS, 0.1, alpha=2.5, delta=1e-3)
    a = O.step_nd([px, py], q, 12)
    b = O.step_nd([py, px], q.T.copy(), 12)
    assert np.array_equal(a, b.T)
    for sh in [(3, 0), (0, 5), (7, 9)]:
        t = O.step_nd([px, py], np.roll(q, sh, axis=(0, 1)), 12)
        assert np.array_equal(t, np.roll(a, sh, axis=(0, 1)))
    q3 = rng.integers(-500, 500, size=(3, 4, 5))
    ax3 = [P(O.BURGERS_EO, 0.1, delta=1e-3), P(O.BURGERS_EO, 0.2, O.OUTFLOW, delta=1e-3),
           P(O.BURGERS_EO, 0.15, delta=1e-3)]
    a3 = O.step_nd(ax3, q3, 6)
    # swap numpy axes 0 and 2 (directions 2 and 0)
    b3 = O.step_nd([ax3[2], ax3[1], ax3[0]], np.transpose(q3, (2, 1, 0)).copy(), 6)
    assert np.array_equal(a3, np.transpose(b3, (2, 1, 0)))


def test_nd_range_checks():
    # the mirror image of the counterexample above, next to the int32 maximum
    # M = 2^31 - 1: the centre 2^31 - 4 sends 2 * 2^30 - 4 and receives
    # rint(M/2) = 2^30 from each of its two upwind neighbours, ending at 2^31
    M = 2 ** 31 - 1
    q = np.full((4, 4), M, dtype=np.int64)
    q[1, 1] = M - 3
    ax64 = [P(O.UPWIND, 0.5, a=1.0, width=64), P(O.UPWIND, 0.5, a=1.0, width=64)]
    assert O.step_nd(ax64, q, 1)[1, 1] == 2 ** 31
    ax32 = [P(O.UPWIND, 0.5, a=1.0, width=32), P(O.UPWIND, 0.5, a=1.0, width=32)]
    with pytest.raises(O.OracleError):
        O.step_nd(ax32, q, 1)
