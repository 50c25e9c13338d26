"""Oracle pins: interface recovery (Sec. 3.2).

  * the paper's worked example: piecewise-constant states and f = 3/4 give the
    interface gradient (u+ - u-)/h along the normal (golden fixture);
  * for every order, piecewise constants give a closed-form gradient
    c(n, f) (u+ - u-)/h computed with numpy's Legendre integrals;
  * the recovered polynomial has order n+1 along the normal and reproduces any
    global polynomial of degree <= n exactly, value and full gradient;
  * the recovered value of piecewise constants is the average (u- + u+)/2.
"""
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _worked_example():
    with open(os.path.join(GOLDEN, "recovery_example.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                f, c = map(float, line.split())
                return f, c


def _const_cells(prob, uL, uR):
    F, M = prob.nfields, prob.nmodes
    wL = np.zeros((F, M))
    wR = np.zeros((F, M))
    wL[:, 0] = uL
    wR[:, 0] = uR
    return wL, wR


def _step_gradient_coefficient(order):
    """Closed form of the recovered normal gradient of piecewise constants,
    grad = c (u+ - u-)/h: projecting the step (u+ - u-)/2 sign(xi*) onto the
    degree-(n+1) Legendre basis gives
    c = (1/(2f)) sum_{odd l <= n+1} (2l+1) (int_0^1 P_l) P_l'(0),
    evaluated here with numpy's Legendre routines."""
    L = np.polynomial.legendre
    f = 0.75 if order - 1 <= 2 else 1.0
    c = 0.0
    for l in range(1, order + 1, 2):
        e = np.zeros(l + 1)
        e[l] = 1.0
        I = L.legval(1.0, L.legint(e)) - L.legval(0.0, L.legint(e))
        c += (2 * l + 1) * I * L.legval(0.0, L.legder(e))
    return c / (2 * f)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("dim", [2, 3])
def test_worked_example_f_three_quarters(order, dim):
    """The paper's example: f = 3/4, piecewise constants -> (u+ - u-)/h.  Exact
    for n = 0 (and n = 1, where the added quadratic has zero slope at the face)."""
    f, coeff = _worked_example()
    assert O.recovery_fraction(order) == f
    h = 0.1
    prob = O.Problem(dim, (4,) * dim, h, order, 1.4, nu=1e-3)
    uL = np.arange(1, prob.nfields + 1, dtype=float)
    uR = uL * 1.7 + 0.3
    for a in range(dim):
        wL, wR = _const_cells(prob, uL, uR)
        ut, gt = prob.recover_face(wL, wR, a)
        np.testing.assert_allclose(gt[:, a, :], np.broadcast_to(coeff * (uR - uL) / h, gt[:, a, :].shape),
                                   rtol=1e-12)
        np.testing.assert_allclose(ut, np.broadcast_to(0.5 * (uL + uR), ut.shape), rtol=1e-13)
        for b in range(dim):
            if b != a:
                np.testing.assert_allclose(gt[:, b, :], 0.0, atol=1e-10)


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5, 8])
def test_piecewise_constant_closed_form(order):
    h = 0.05
    prob = O.Problem(2, (4, 4), h, order, 1.4, nu=1e-3)
    uL = np.array([1.0, 0.2, -0.3, 2.0])
    uR = np.array([0.5, 0.1, 0.4, 1.0])
    wL, wR = _const_cells(prob, uL, uR)
    c = _step_gradient_coefficient(order)
    for a in range(2):
        ut, gt = prob.recover_face(wL, wR, a)
        np.testing.assert_allclose(gt[:, a, :], np.broadcast_to(c * (uR - uL) / h, gt[:, a, :].shape),
                                   rtol=1e-12)
        np.testing.assert_allclose(ut, np.broadcast_to(0.5 * (uL + uR), ut.shape), rtol=1e-13)
    if order <= 2:
        assert abs(c - 1.0) < 1e-14


def _project_poly(order, coeffs_fn, xc, h, dim, nfields):
    """Modal coefficients of a polynomial on the cell centred at xc, by a
    high-order Gauss rule (numpy)."""
    x, wq = np.polynomial.legendre.leggauss(order + 4)
    V = np.polynomial.legendre.legvander(x, order - 1) * np.sqrt(2 * np.arange(order) + 1)
    M = order ** dim
    out = np.zeros((nfields, M))
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    pts = [xc[a] + 0.5 * h * grids[a] for a in range(dim)]
    vals = coeffs_fn(*pts)          # (nfields, q, q[, q]) with axis a = dim a
    Wt = 0.5 * wq
    for m in range(M):
        l = [(m // order ** a) % order for a in range(dim)]
        phiw = np.ones_like(grids[0])
        for a in range(dim):
            shape = [1] * dim
            shape[a] = -1
            phiw = phiw * (Wt * V[:, l[a]]).reshape(shape)
        out[:, m] = (vals * phiw[None]).reshape(nfields, -1).sum(axis=1)
    return out


@pytest.mark.parametrize("order", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_polynomial_reproduction_3d(order, axis):
    n = order - 1
    h = 0.2
    dim = 3
    prob = O.Problem(dim, (4, 4, 4), h, order, 1.4, nu=1e-3)
    F = prob.nfields
    rng = np.random.default_rng(order * 10 + axis)
    # per field a random polynomial of degree <= n in each variable
    C = rng.standard_normal((F, n + 1, n + 1, n + 1))

    def poly(x, y, z):
        out = np.zeros((F,) + np.shape(x))
        for f in range(F):
            for i in range(n + 1):
                for j in range(n + 1):
                    for k in range(n + 1):
                        out[f] += C[f, i, j, k] * x ** i * y ** j * z ** k
        return out

    def dpoly(x, y, z, b):
        out = np.zeros((F,) + np.shape(x))
        for f in range(F):
            for i in range(n + 1):
                for j in range(n + 1):
                    for k in range(n + 1):
                        e = [i, j, k]
                        if e[b] == 0:
                            continue
                        t = C[f, i, j, k] * e[b]
                        e[b] -= 1
                        out[f] += t * x ** e[0] * y ** e[1] * z ** e[2]
        return out

    xf = np.zeros(3)                    # the face sits at the origin
    xcL = xf.copy()
    xcL[axis] -= 0.5 * h
    xcR = xf.copy()
    xcR[axis] += 0.5 * h
    wL = _project_poly(order, poly, xcL, h, dim, F)
    wR = _project_poly(order, poly, xcR, h, dim, F)
    ut, gt = prob.recover_face(wL, wR, axis)
    xg, _ = np.polynomial.legendre.leggauss(order)
    tdims = [b for b in range(3) if b != axis]
    K = order ** 2
    for k in range(K):
        pt = np.zeros(3)
        pt[tdims[0]] = 0.5 * h * xg[k % order]
        pt[tdims[1]] = 0.5 * h * xg[k // order]
        ref = poly(*pt)
        np.testing.assert_allclose(ut[k], ref, rtol=1e-11, atol=1e-11)
        for b in range(3):
            np.testing.assert_allclose(gt[k, b], dpoly(*pt, b), rtol=1e-9, atol=1e-9)
