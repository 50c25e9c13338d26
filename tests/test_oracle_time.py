"""Oracle pins for time stepping (Sec. 2.5) and whole-run behaviour (Sec. 5).

  * temporal order of the SSP-RK schemes on a nonlinear problem: 2 for p = 2,
    3 for p = 3, 4 for p >= 4 (the 5-stage 4th-order scheme);
  * linear stability polynomial R(z) agrees with e^z to the scheme's order;
  * CFL step eq. timestep in closed form for a uniform state;
  * conserved totals of a uniform state;
  * the 2D density-wave run (uniform v, P) equals R(dt A)^N w0 with A the
    exact-integral upwind advection operator and R the SSPRK(3,3) polynomial;
  * density-wave error falls with order p (exponential convergence, Sec. 5.1);
  * viscous shear-wave decay v_y = A exp(-4 pi^2 nu t) sin 2 pi x converges at
    order p (diffusion convergence claim of Sec. 5.2);
  * Sod tube with artificial viscosity converges in L1 to the exact Riemann
    solution (first order for a discontinuous solution).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2208_11131_amd import workloads as W
from tests import refsol


def _run(prob, w, dt, nsteps, R=None):
    for _ in range(nsteps):
        w, R = prob.step(w, dt, R)
    return w, R


@pytest.mark.parametrize("order,expect", [(2, 2), (3, 3), (4, 4)])
def test_temporal_order(order, expect):
    # supersonic mean flow along (1,1): every face takes the upwind HLLC
    # branch, so the RHS is a smooth nonlinear function of the state
    n = (3, 3)
    prob = O.Problem(2, n, 0.5, order, 1.4, nu=2e-3, kappa=2e-3)
    w0 = W.random_smooth(2, n, order, seed=11, amp=0.05, vbase=(3.0, 3.0)).numpy()
    T = 0.016
    ref, _ = _run(prob, w0, T / 128, 128)
    errs = []
    for N in (8, 16):
        w, _ = _run(prob, w0, T / N, N)
        errs.append(np.abs(w - ref).max())
    rate = math.log2(errs[0] / errs[1])
    assert abs(rate - expect) < 0.35, (errs, rate)


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_linear_stability_polynomial(order):
    """Pure decay dalpha/dt = -lambda alpha (quiescent AV field): one step gives
    R(z) alpha0 with z = -lambda dt; R agrees with e^z through z^q."""
    q = {1: 1, 2: 2, 3: 3, 4: 4}[order]
    h = 0.1
    prob = O.Problem(2, (2, 2), h, order, 1.4, av={"f_tau": 0.5})
    w = np.zeros(prob.shape)
    w[:, 0, 0] = 1.0
    w[:, 3, 0] = 1.0 / 0.4
    w[:, 4, 0] = 1.0
    lam = order * math.sqrt(1.4) / (0.5 * h)
    for z in (-0.05, -0.1):
        w1, _ = prob.step(w, -z / lam, np.zeros(prob.ncells))
        R = w1[0, 4, 0]
        taylor = sum(z ** k / math.factorial(k) for k in range(q + 1))
        # remainder is O(z^(q+1)); the (q+1)-th coefficient is at most 1/(q+1)!
        assert abs(R - taylor) <= 1.05 * abs(z) ** (q + 1) / math.factorial(q + 1) + 1e-15
        if q < 4:
            # schemes with S = q stages are exactly the Taylor polynomial
            assert abs(R - taylor) < 1e-14
        # and the other fields are untouched
        np.testing.assert_allclose(w1[:, :4], w[:, :4], rtol=0, atol=1e-14)


def test_cfl_closed_form():
    g = 1.4
    prob = O.Problem(3, (2, 2, 2), 0.1, 3, g, cfl=0.3)
    w = np.zeros(prob.shape)
    rho, v, P = 1.7, np.array([0.3, -0.4, 1.2]), 2.3
    w[:, 0, 0] = rho
    w[:, 1:4, 0] = rho * v
    w[:, 4, 0] = P / (g - 1) + 0.5 * rho * v @ v
    dt, cm, vm = prob.max_dt(w)
    cs = math.sqrt(g * P / rho)
    assert abs(cm - cs) < 1e-14 and abs(vm - np.linalg.norm(v)) < 1e-14
    assert abs(dt - 0.3 * 0.1 / (2 * 3 * (cs + np.linalg.norm(v)))) < 1e-16


def test_cfl_maximum_over_gauss_points():
    """With a linear density profile inside a cell, c_s peaks at the Gauss
    point of lowest density (not at the cell edge, not at the mean)."""
    g = 1.4
    order = 3
    prob = O.Problem(2, (1, 1), 1.0, order, g)
    w = np.zeros(prob.shape)
    w[0, 0, 0] = 1.0
    w[0, 0, 1] = 0.2                          # rho = 1 + 0.2 sqrt(3) xi_x
    w[0, 3, 0] = 1.0 / (g - 1)                # P = 1, v = 0
    dt, cm, vm = prob.max_dt(w)
    x, _ = np.polynomial.legendre.leggauss(order)
    rmin = 1.0 + 0.2 * math.sqrt(3) * x.min()
    assert abs(cm - math.sqrt(g / rmin)) < 1e-14 and vm == 0.0


def test_totals_uniform():
    prob = O.Problem(2, (5, 3), 0.2, 2, 1.4)
    w = np.zeros(prob.shape)
    w[:, :, 0] = [1.5, 0.25, -0.5, 3.0]
    w[:, :, 1:] = 7.0                          # higher modes have zero mean
    tot = prob.totals(w)
    np.testing.assert_allclose(tot, np.array([1.5, 0.25, -0.5, 3.0]) * 15 * 0.04, rtol=1e-15)


def test_density_wave_closed_form_run():
    """Full-run closed form of the 2D density wave: w(t_N) = R(dt A)^N w0 with
    R(z) = 1 + z + z^2/2 + z^3/6 (SSPRK(3,3)) and A the exact upwind operator."""
    order, n = 3, 16
    h = 1.0 / n
    w0 = W.density_wave(order, n).numpy()
    prob = O.Problem(2, (n, n), h, order, 5.0 / 3.0, cfl=0.3)
    dt, _, _ = prob.max_dt(w0)
    N = 20
    w, _ = _run(prob, w0, dt, N)
    A = refsol.upwind_advection_operator(order, n, h)
    for f in range(4):
        x = w0[:, f, :].reshape(-1).copy()
        for _ in range(N):
            y1 = dt * (A @ x)
            y2 = dt * (A @ y1)
            y3 = dt * (A @ y2)
            x = x + y1 + y2 / 2 + y3 / 6
        np.testing.assert_allclose(w[:, f, :].reshape(-1), x, rtol=0, atol=1e-12 * np.abs(x).max())


def test_density_wave_error_falls_with_order():
    n, T = 6, 0.05
    errs = []
    for order in (1, 2, 3, 4, 5):
        w0 = W.density_wave(order, n).numpy()
        prob = O.Problem(2, (n, n), 1.0 / n, order, 5.0 / 3.0, cfl=0.3)
        dt, _, _ = prob.max_dt(w0)
        N = int(math.ceil(T / dt))
        w, _ = _run(prob, w0, T / N, N)
        ex = W.density_wave_exact(order, n, T).numpy()
        errs.append(np.sqrt(((w[:, 0] - ex[:, 0]) ** 2).sum() / w.shape[0]))
    for i in range(len(errs) - 1):
        assert errs[i + 1] < 0.5 * errs[i], errs


@pytest.mark.parametrize("order,ns,rate_min", [(2, (8, 16, 32), 1.7), (3, (8, 16, 32), 2.0),
                                               (4, (4, 8, 16), 3.7)])
def test_shear_wave_decay_converges(order, ns, rate_min):
    """v_y = A exp(-4 pi^2 nu t) sin 2 pi x with uniform rho and P is an exact
    solution of the momentum equation.  Observed rates: about p for p = 2, 4;
    about 2.3 for p = 3, where the prescribed overlap f = 3/4 (n <= 2) limits
    the recovered gradient's accuracy (f = 1 would give 3)."""
    nu, A, T, g = 0.005, 1e-3, 0.2, 1.4

    def ic(t):
        def fn(X):
            x, y = X
            one = torch.ones_like(x)
            vy = A * math.exp(-4 * math.pi ** 2 * nu * t) * torch.sin(2 * math.pi * x)
            return W._conserved(one, [0 * x, vy], one, g)
        return fn

    errs = []
    for n in ns:
        h = 1.0 / n
        w0 = W.project(ic(0.0), 2, (n, 1), (0.0, 0.0), h, order).numpy()
        prob = O.Problem(2, (n, 1), h, order, g, nu=nu)
        dt, _, _ = prob.max_dt(w0)
        N = int(math.ceil(T / dt))
        w, _ = _run(prob, w0, T / N, N)
        ex = W.project(ic(T), 2, (n, 1), (0.0, 0.0), h, order).numpy()
        errs.append(np.sqrt(((w[:, 2] - ex[:, 2]) ** 2).sum() / n) / A)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] > rate_min, (errs, rates)


@pytest.mark.slow
@pytest.mark.parametrize("order", [2, 4])
def test_sod_l1_converges_to_exact_riemann(order):
    """Sod tube (gamma = 1.4, t = 0.2) with the AV defaults on a 1-cell deep
    strip: L1(rho) against the exact solution falls roughly like 1/N."""
    T, g = 0.2, 1.4
    av = {}
    errs = []
    for nx in (32, 64):
        h = 1.0 / nx
        w0 = W.sod(order, nx, 1).numpy()
        prob = O.Problem(2, (nx, 1), h, order, g, av=av, bc=(2, 0), cfl=0.3)
        t, R = 0.0, np.zeros(prob.ncells)
        w = w0
        while t < T - 1e-12:
            dt, _, _ = prob.max_dt(w)
            dt = min(dt, T - t)
            w, R = prob.step(w, dt, R)
            t += dt
        xq, wq = np.polynomial.legendre.leggauss(order + 2)
        V = np.polynomial.legendre.legvander(xq, order - 1) * np.sqrt(2 * np.arange(order) + 1)
        rho_q = w[:, 0, :order] @ V.T                  # y-uniform: modes l_y = 0
        xc = (np.arange(nx) + 0.5) * h
        X = (xc[:, None] + 0.5 * h * xq[None, :]).reshape(-1)
        ex = refsol.exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, g, (X - 0.5) / T)[0].reshape(nx, -1)
        errs.append(float((np.abs(rho_q - ex) * 0.5 * wq[None, :]).sum() * h))
        assert np.all(np.isfinite(w))
    assert errs[0] < 0.02 and errs[1] < 0.7 * errs[0], errs
