"""Exact solutions used as independent references -- TEST INFRASTRUCTURE.

* :func:`shift` -- exact solution of linear advection, u0(x - a t) on the
  periodic unit interval (Sec. 3.1 compares against the exact shift).
* :func:`hopf_lax_burgers` -- the entropy solution of inviscid Burgers from the
  Lax-Oleinik (Hopf-Lax) minimisation over a dense auxiliary grid of candidate
  foot points y (Sec. 3.2 uses such a dense-grid entropy reference).
* :func:`riemann_exact` -- the exact Riemann solver of the 1D Euler equations
  for an ideal gas (the exact Sod reference of Sec. 3.3), the standard
  pressure-function construction (Toro, Riemann Solvers and Numerical Methods
  for Fluid Dynamics, ch. 4), written from that construction.
"""
from __future__ import annotations

import math

import numpy as np


def shift(u0, x, t, a=1.0):
    """Exact periodic shift u0(x - a t) for u0 a callable on [0, 1)."""
    return u0(np.mod(x - a * t, 1.0))


# --------------------------------------------------------------------------
# Burgers: Lax-Oleinik formula u(x,t) = (x - y*)/t, y* = argmin_y G(y),
# G(y) = U0(y) + (x - y)^2 / (2 t), with U0' = u0.  For a 1-periodic u0 with
# mean M the primitive satisfies U0(y + 1) = U0(y) + M.
# --------------------------------------------------------------------------
class SineStepData:
    """u0(x) = b + A sin(2 pi m x + theta) + h 1[x >= xs] on [0, 1), periodic."""

    def __init__(self, b=0.5, A=1.0, m=1, theta=0.0, h=0.0, xs=0.0):
        self.b, self.A, self.m, self.theta, self.h, self.xs = b, A, m, theta, h, xs

    def u0(self, x):
        x = np.mod(x, 1.0)
        return (self.b + self.A * np.sin(2 * np.pi * self.m * x + self.theta)
                + self.h * (x >= self.xs))

    def mean(self):
        return self.b + self.h * (1.0 - self.xs)

    def primitive(self, y):
        y = np.asarray(y, dtype=np.float64)
        k = np.floor(y)
        f = y - k
        w = 2 * np.pi * self.m
        U = (self.b * f + self.A * (np.cos(self.theta) - np.cos(w * f + self.theta)) / w
             + self.h * np.maximum(f - self.xs, 0.0))
        return k * self.mean() + U

    def bounds(self):
        lo = self.b - abs(self.A) + min(self.h, 0.0)
        hi = self.b + abs(self.A) + max(self.h, 0.0)
        return lo, hi


def hopf_lax_burgers(data: SineStepData, x, t, ny=2048, refine=True):
    """Entropy solution of u_t + (u^2/2)_x = 0 at points x and time t > 0.

    For each x the foot point is searched on ``ny`` candidates spanning the
    window [x - t*max u0, x - t*min u0] (outside it G cannot be minimal), then
    refined by golden-section search on the bracketing cell when ``refine``.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    lo, hi = data.bounds()
    out = np.empty_like(x)
    s = np.linspace(0.0, 1.0, ny)
    for j, xj in enumerate(x):
        ya, yb = xj - t * hi, xj - t * lo
        y = ya + (yb - ya) * s
        G = data.primitive(y) + (xj - y) ** 2 / (2 * t)
        k = int(np.argmin(G))
        ys = y[k]
        if refine and ny > 2:
            a = y[max(k - 1, 0)]
            b = y[min(k + 1, ny - 1)]
            g = (math.sqrt(5) - 1) / 2
            c, d = b - g * (b - a), a + g * (b - a)

            def Gf(v):
                return float(data.primitive(v) + (xj - v) ** 2 / (2 * t))

            fc, fd = Gf(c), Gf(d)
            for _ in range(80):
                if fc < fd:
                    b, d, fd = d, c, fc
                    c = b - g * (b - a)
                    fc = Gf(c)
                else:
                    a, c, fc = c, d, fd
                    d = a + g * (b - a)
                    fd = Gf(d)
            ym = 0.5 * (a + b)
            if Gf(ym) <= G[k]:
                ys = ym
        out[j] = (xj - ys) / t
    return out


# --------------------------------------------------------------------------
# Exact Riemann solver for the Euler equations, ideal gas with ratio gamma.
# --------------------------------------------------------------------------
def _pressure_function(p, rho, pK, cK, g):
    """f_K(p) and its derivative (Toro eq. 4.6-4.7 in structure)."""
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        sq = math.sqrt(A / (p + B))
        return (p - pK) * sq, sq * (1.0 - 0.5 * (p - pK) / (B + p))
    # rarefaction
    r = p / pK
    f = 2.0 * cK / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * cK) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, gamma=1.4, tol=1e-14):
    """Star-region pressure and velocity for left/right (rho, u, p)."""
    rL, uL, pL = left
    rR, uR, pR = right
    g = gamma
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    du = uR - uL
    if 2.0 * (cL + cR) / (g - 1.0) <= du:
        raise ValueError("vacuum is generated")
    p = max(0.5 * (pL + pR) - 0.125 * du * (rL + rR) * (cL + cR), 1e-12)
    for _ in range(200):
        fL, dL = _pressure_function(p, rL, pL, cL, g)
        fR, dR = _pressure_function(p, rR, pR, cR, g)
        pn = p - (fL + fR + du) / (dL + dR)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _pressure_function(p, rL, pL, cL, g)
    fR, _ = _pressure_function(p, rR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def riemann_exact(left, right, xi, gamma=1.4):
    """Exact self-similar solution (rho, u, p) at xi = (x - x0)/t."""
    rL, uL, pL = left
    rR, uR, pR = right
    g = gamma
    ps, us = star_state(left, right, g)
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for j, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pL:  # left shock
                rs = rL * ((ps / pL + gm) / (gm * ps / pL + 1.0))
                SL = uL - cL * math.sqrt((g + 1.0) / (2 * g) * ps / pL + (g - 1.0) / (2 * g))
                st = (rL, uL, pL) if s <= SL else (rs, us, ps)
            else:  # left rarefaction
                cs = cL * (ps / pL) ** ((g - 1.0) / (2 * g))
                SH, ST = uL - cL, us - cs
                if s <= SH:
                    st = (rL, uL, pL)
                elif s >= ST:
                    st = (rL * (ps / pL) ** (1.0 / g), us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * uL + s)
                    cc = 2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * (uL - s))
                    rr = rL * (cc / cL) ** (2.0 / (g - 1.0))
                    st = (rr, uu, pL * (cc / cL) ** (2.0 * g / (g - 1.0)))
        else:  # right of contact
            if ps > pR:  # right shock
                rs = rR * ((ps / pR + gm) / (gm * ps / pR + 1.0))
                SR = uR + cR * math.sqrt((g + 1.0) / (2 * g) * ps / pR + (g - 1.0) / (2 * g))
                st = (rR, uR, pR) if s >= SR else (rs, us, ps)
            else:  # right rarefaction
                cs = cR * (ps / pR) ** ((g - 1.0) / (2 * g))
                SH, ST = uR + cR, us + cs
                if s >= SH:
                    st = (rR, uR, pR)
                elif s <= ST:
                    st = (rR * (ps / pR) ** (1.0 / g), us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (-cR + (g - 1.0) / 2.0 * uR + s)
                    cc = 2.0 / (g + 1.0) * (cR - (g - 1.0) / 2.0 * (uR - s))
                    rr = rR * (cc / cR) ** (2.0 / (g - 1.0))
                    st = (rr, uu, pR * (cc / cR) ** (2.0 * g / (g - 1.0)))
        rho[j], u[j], p[j] = st
    return rho, u, p


def shock_speed_right(left, right, gamma=1.4):
    """Speed of the right-going shock (when the right wave is a shock)."""
    rR, uR, pR = right
    ps, _ = star_state(left, right, gamma)
    g = gamma
    cR = math.sqrt(g * pR / rR)
    return uR + cR * math.sqrt((g + 1.0) / (2 * g) * ps / pR + (g - 1.0) / (2 * g))
