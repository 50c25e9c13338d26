"""Oracle pins of the positivity limiter (Sec. 4.2).

Checked against values computed here independently (numpy Legendre values at
the limiter points, closed forms of the scale factors):
  * the point set is the volume Gauss points plus the Gauss points of the
    cell's faces: a density dip at a face point triggers the limiter, a dip
    at a corner alone does not;
  * density: every weight of degree >= 1 of every field is multiplied by
    theta = (rho_bar - rho_bottom) / (rho_bar - rho_min), rho_bottom =
    1e-6 rho_bar, so the minimum over the points becomes rho_bottom; cell
    means are kept;
  * pressure: the higher weights are halved until the pressure at every
    point is >= 1e-6 p_bar (the number of halvings in closed form for a gas
    at rest, where p is linear in the weights);
  * cells that need nothing are untouched; cells with a non-positive mean are
    left to the error check;
  * whole steps with the limiter keep every stage state positive at the
    limiter points, where the same steps without it break down (negative
    pressure, non-finite weights).
"""
import math

import numpy as np
import pytest

import oracle as O

G = 1.4


def leg_t(order, x):
    """Pt_l(x) = sqrt(2l+1) P_l(x), l < order, at the points x (array)."""
    V = np.polynomial.legendre.legvander(np.asarray(x, dtype=float), order - 1)
    return V * np.sqrt(2 * np.arange(order) + 1)


def limiter_points(order, dim):
    xg, _ = np.polynomial.legendre.leggauss(order)
    pts = [np.array(t) for t in np.stack(np.meshgrid(*([xg] * dim), indexing="ij"), -1).reshape(-1, dim)]
    for a in range(dim):
        for side in (-1.0, 1.0):
            for t in np.stack(np.meshgrid(*([xg] * (dim - 1)), indexing="ij"), -1).reshape(-1, dim - 1):
                x = np.insert(t, a, side)
                pts.append(x)
    return np.array(pts)


def values(wc, order, dim, pts):
    """Field values (F, npts) of one cell's coefficients wc (F, order^dim)."""
    M = order ** dim
    phi = np.ones((len(pts), M))
    for m in range(M):
        r = m
        for a in range(dim):
            l = r % order
            r //= order
            phi[:, m] *= leg_t(order, pts[:, a])[:, l]
    return wc @ phi.T


def pressure(u, dim):
    rho = u[0]
    ke = 0.5 * sum(u[1 + i] ** 2 for i in range(dim)) / rho
    return (G - 1) * (u[dim + 1] - ke)


def one_cell(dim, order, F=None):
    F = F or dim + 2
    prob = O.Problem(dim, (1,) * dim, 1.0, order, G)
    w = np.zeros((1, F, order ** dim))
    return prob, w


def mode(order, dim, l):
    m = 0
    for a in reversed(range(dim)):
        m = m * order + l[a]
    return m


@pytest.mark.parametrize("dim,order", [(2, 4), (3, 3), (2, 6)])
def test_density_scaling(dim, order):
    prob, w = one_cell(dim, order)
    rng = np.random.default_rng(order)
    w[0, 0, 0] = 1.0
    w[0, 0, 1:] = 0.6 * rng.standard_normal(order ** dim - 1)
    # no momentum (a near-vacuum point would otherwise carry a large kinetic
    # energy and trigger the pressure stage as well)
    w[0, dim + 1, 0] = 50.0
    w[0, dim + 1, 1:] = 0.01 * rng.standard_normal(order ** dim - 1)
    pts = limiter_points(order, dim)
    rmin = values(w[0], order, dim, pts)[0].min()
    assert rmin < 0.0
    wl, n = prob.limit(w)
    assert n == 1
    theta = (1.0 - 1e-6) / (1.0 - rmin)
    np.testing.assert_array_equal(wl[0, :, 0], w[0, :, 0])
    np.testing.assert_allclose(wl[0, :, 1:], theta * w[0, :, 1:], rtol=1e-13, atol=0)
    new_min = values(wl[0], order, dim, pts)[0].min()
    assert abs(new_min - 1e-6) <= 1e-13


def test_face_point_dip_triggers_corner_dip_does_not():
    dim, order = 2, 4
    n = order - 1                                    # odd degree: Pt_n(-1) = -sqrt(2n+1)
    pts = limiter_points(order, dim)
    # 1. a dip at the face xi_x = -1 only (the Gauss points stay positive)
    prob, w = one_cell(dim, order)
    w[0, 0, 0] = 1.0
    w[0, 0, mode(order, dim, (n, 0))] = 1.2 / math.sqrt(2 * n + 1)
    w[0, 3, 0] = 10.0
    xg, _ = np.polynomial.legendre.leggauss(order)
    vol = values(w[0], order, dim, np.stack(np.meshgrid(xg, xg, indexing="ij"), -1).reshape(-1, 2))[0]
    assert vol.min() > 0.5
    assert values(w[0], order, dim, pts)[0].min() < -0.1
    wl, nchg = prob.limit(w)
    assert nchg == 1 and values(wl[0], order, dim, pts)[0].min() >= 1e-6 * (1 - 1e-12)
    # 2. a dip at the corner (-1, 1) only
    prob, w = one_cell(dim, order)
    w[0, 0, 0] = 1.0
    w[0, 0, mode(order, dim, (n, n))] = 0.3
    w[0, 3, 0] = 10.0
    corner = values(w[0], order, dim, np.array([[-1.0, 1.0]]))[0, 0]
    assert corner < -1.0
    assert values(w[0], order, dim, pts)[0].min() > 0.1
    wl, nchg = prob.limit(w)
    assert nchg == 0
    np.testing.assert_array_equal(wl, w)


@pytest.mark.parametrize("dim,order", [(2, 5), (3, 2)])
def test_pressure_halving_count(dim, order):
    """Gas at rest (zero momentum), uniform density: p = (gamma-1) E is linear
    in the weights, so p_min(theta) = p_bar + theta (p_min - p_bar) and the
    number of halvings is the smallest k with p_bar + 2^-k (p_min - p_bar)
    >= 1e-6 p_bar."""
    prob, w = one_cell(dim, order)
    rng = np.random.default_rng(3)
    w[0, 0, 0] = 1.0
    w[0, dim + 1, 0] = 2.0
    w[0, dim + 1, 1:] = 1.5 * rng.standard_normal(order ** dim - 1)
    pts = limiter_points(order, dim)
    pv = pressure(values(w[0], order, dim, pts), dim)
    pbar = (G - 1) * 2.0
    pmin = pv.min()
    assert pmin < 0.0
    k = 0
    while pbar + 2.0 ** -k * (pmin - pbar) < 1e-6 * pbar:
        k += 1
    wl, nchg = prob.limit(w)
    assert nchg == 1
    np.testing.assert_array_equal(wl[0, :, 0], w[0, :, 0])
    np.testing.assert_allclose(wl[0, dim + 1, 1:], 2.0 ** -k * w[0, dim + 1, 1:], rtol=1e-15, atol=0)


def test_untouched_cells():
    dim, order = 2, 4
    prob, w = one_cell(dim, order)
    rng = np.random.default_rng(9)
    w[0, 0, 0] = 1.0
    w[0, 0, 1:] = 0.01 * rng.standard_normal(order ** dim - 1)
    w[0, 3, 0] = 3.0
    wl, nchg = prob.limit(w)
    assert nchg == 0
    np.testing.assert_array_equal(wl, w)
    # a non-positive mean density is left to the error check
    w2 = w.copy()
    w2[0, 0, 0] = -0.1
    w2[0, 0, 1] = 1.0
    wl, nchg = prob.limit(w2)
    assert nchg == 0
    np.testing.assert_array_equal(wl, w2)


def _blast(order, nx):
    """Strong two-state tube along x (density 1 : 1e-3, pressure 1 : 1e-5),
    the jump inside cell nx/2 at a third of its width: its projection on the
    basis undershoots below zero (Gibbs) at the start."""
    F = 4
    M = order * order
    w = np.zeros((nx, F, M))
    left = np.arange(nx) < nx // 2
    w[:, 0, 0] = np.where(left, 1.0, 1e-3)
    w[:, 3, 0] = np.where(left, 1.0, 1e-5) / (G - 1)
    c, x0 = nx // 2, -1.0 / 3.0
    w[c] = 0.0
    xq, wq = np.polynomial.legendre.leggauss(40)
    for lo, hi, val in ((-1.0, x0, (1.0, 1.0 / (G - 1))), (x0, 1.0, (1e-3, 1e-5 / (G - 1)))):
        x = 0.5 * (hi - lo) * xq + 0.5 * (hi + lo)
        wt = 0.5 * (hi - lo) * wq
        P = leg_t(order, x)                          # (q, l), y-uniform modes l_y = 0
        for f, v in ((0, val[0]), (3, val[1])):
            w[c, f, :order] += 0.5 * v * (wt[:, None] * P).sum(axis=0)
    return w


def test_steps_keep_stage_states_positive():
    order, nx = 6, 16
    h = 1.0 / nx
    pts = limiter_points(order, 2)

    def min_point_values(w):
        assert np.isfinite(w).all()
        rmin, pmin = np.inf, np.inf
        for c in range(nx):
            u = values(w[c], order, 2, pts)
            rb, pb = w[c, 0, 0], pressure(w[c, :, 0:1], 2)[0]
            rmin = min(rmin, (u[0] / rb).min())
            pmin = min(pmin, (pressure(u, 2) / pb).min())
        return rmin, pmin

    w0 = _blast(order, nx)
    on = O.Problem(2, (nx, 1), h, order, G, bc=(2, 0), cfl=0.3, limiter=True)
    off = O.Problem(2, (nx, 1), h, order, G, bc=(2, 0), cfl=0.3)
    # the initial projection undershoots: it is limited once before stepping
    # (the steps limit every state they produce)
    wl, nchg = on.limit(w0)
    assert nchg >= 1
    dt = on.max_dt(wl)[0]
    wa, wb = wl, w0
    worst_off = np.inf
    for _ in range(3):
        wa, _ = on.step(wa, dt)
        wb, _ = off.step(wb, dt)
        ra, pa = min_point_values(wa)
        assert ra >= 1e-6 * (1 - 1e-9) and pa >= 1e-6 * (1 - 1e-9), (ra, pa)
        if np.isfinite(wb).all():
            worst_off = min(worst_off, min(min_point_values(wb)))
        else:
            worst_off = -np.inf                      # the unlimited run broke down
    assert worst_off < 0.0
    # the limiter keeps every cell mean of the final state of its own stages:
    # the totals are conserved with walls on the x ends
    assert abs(wa[:, 0, 0].sum() - w0[:, 0, 0].sum()) <= 1e-13 * w0[:, 0, 0].sum()
