"""Independent reference solutions used to pin the oracle (test helpers).

  * ``upwind_advection_operator``: the DG operator of scalar linear advection
    with constant velocity (a, b) > 0 and upwind flux on a periodic 2D grid,
    built from exact polynomial integrals (numpy.polynomial.legendre), not from
    quadrature.  For a flow with uniform velocity and pressure the Euler
    equations reduce to this advection for every conserved field, and HLLC
    reduces to upwinding at such a contact.
  * ``exact_riemann``: the exact solution of the 1D Riemann problem for an
    ideal gas (Toro, Riemann Solvers and Numerical Methods, ch. 4), written
    from the textbook's pressure-function formulation.
"""
import math

import numpy as np
from numpy.polynomial import legendre as L


def _scaled(l):
    c = np.zeros(l + 1)
    c[l] = math.sqrt(2 * l + 1)
    return c


def stiffness_1d(order):
    """S[l, m] = (1/2) int_{-1}^{1} Pt_l'(x) Pt_m(x) dx, exact."""
    S = np.zeros((order, order))
    for l in range(order):
        for m in range(order):
            prod = L.legmul(L.legder(_scaled(l)), _scaled(m))
            I = L.legint(prod)
            S[l, m] = 0.5 * (L.legval(1.0, I) - L.legval(-1.0, I))
    return S


def endpoint_values(order):
    ep = np.array([L.legval(1.0, _scaled(l)) for l in range(order)])
    em = np.array([L.legval(-1.0, _scaled(l)) for l in range(order)])
    return ep, em


def upwind_advection_operator(order, n, h, a=1.0, b=1.0):
    """Dense matrix A with dw/dt = A w for w[cell][mode] (cell = i + n j,
    mode = l_x + p l_y) on an n x n periodic grid, velocity (a, b) > 0."""
    p = order
    S = stiffness_1d(p)
    ep, em = endpoint_values(p)
    I = np.eye(p)
    # per-cell blocks acting on mode vectors (mode = lx + p ly => kron(Iy, Ax))
    vol = (2 * a / h) * np.kron(I, S) + (2 * b / h) * np.kron(S, I)
    own = -(a / h) * np.kron(I, np.outer(ep, ep)) - (b / h) * np.kron(np.outer(ep, ep), I)
    left = (a / h) * np.kron(I, np.outer(em, ep))
    below = (b / h) * np.kron(np.outer(em, ep), I)
    M = p * p
    N = n * n
    A = np.zeros((N * M, N * M))
    for j in range(n):
        for i in range(n):
            c = i + n * j
            cl = (i - 1) % n + n * j
            cb = i + n * ((j - 1) % n)
            A[c * M:(c + 1) * M, c * M:(c + 1) * M] += vol + own
            A[c * M:(c + 1) * M, cl * M:(cl + 1) * M] += left
            A[c * M:(c + 1) * M, cb * M:(cb + 1) * M] += below
    return A


# ---------------------------------------------------------------------------
# exact Riemann solver (Toro ch. 4)
# ---------------------------------------------------------------------------

def _fK(p, rK, pK, cK, g):
    if p > pK:   # shock
        A = 2.0 / ((g + 1) * rK)
        B = (g - 1) / (g + 1) * pK
        f = (p - pK) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1 - (p - pK) / (2 * (B + p)))
    else:        # rarefaction
        f = 2 * cK / (g - 1) * ((p / pK) ** ((g - 1) / (2 * g)) - 1)
        df = 1.0 / (rK * cK) * (p / pK) ** (-(g + 1) / (2 * g))
    return f, df


def star_state(rL, uL, pL, rR, uR, pR, g):
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    p = max(1e-8, 0.5 * (pL + pR))
    for _ in range(200):
        fL, dL = _fK(p, rL, pL, cL, g)
        fR, dR = _fK(p, rR, pR, cR, g)
        dp = (fL + fR + (uR - uL)) / (dL + dR)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _fK(p, rL, pL, cL, g)
    fR, _ = _fK(p, rR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def exact_riemann(rL, uL, pL, rR, uR, pR, g, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    ps, us = star_state(rL, uL, pL, rR, uR, pR, g)
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    out = np.zeros((3, len(xi)))
    gm = (g - 1) / (g + 1)
    for i, s in enumerate(xi):
        if s <= us:   # left of contact
            if ps > pL:
                SL = uL - cL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                if s <= SL:
                    out[:, i] = (rL, uL, pL)
                else:
                    r = rL * (ps / pL + gm) / (gm * ps / pL + 1)
                    out[:, i] = (r, us, ps)
            else:
                cs = cL * (ps / pL) ** ((g - 1) / (2 * g))
                if s <= uL - cL:
                    out[:, i] = (rL, uL, pL)
                elif s >= us - cs:
                    out[:, i] = (rL * (ps / pL) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (cL + (g - 1) / 2 * uL + s)
                    c = 2 / (g + 1) * (cL + (g - 1) / 2 * (uL - s))
                    r = rL * (c / cL) ** (2 / (g - 1))
                    out[:, i] = (r, u, pL * (c / cL) ** (2 * g / (g - 1)))
        else:
            if ps > pR:
                SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                if s >= SR:
                    out[:, i] = (rR, uR, pR)
                else:
                    r = rR * (ps / pR + gm) / (gm * ps / pR + 1)
                    out[:, i] = (r, us, ps)
            else:
                cs = cR * (ps / pR) ** ((g - 1) / (2 * g))
                if s >= uR + cR:
                    out[:, i] = (rR, uR, pR)
                elif s <= us + cs:
                    out[:, i] = (rR * (ps / pR) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + s)
                    c = 2 / (g + 1) * (cR - (g - 1) / 2 * (uR - s))
                    r = rR * (c / cR) ** (2 / (g - 1))
                    out[:, i] = (r, u, pR * (c / cR) ** (2 * g / (g - 1)))
    return out
