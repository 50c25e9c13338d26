"""Oracle pins of three physics terms by value (CPU only).

  * Driving source (Sec. 7.1): the momentum equation gains rho s and the
    energy equation the work rho s.v, projected with Gauss quadrature.  With
    polynomial fields of degree <= n per axis the projection is exact, so the
    difference L(with s) - L(without s) equals known coefficients exactly.
  * Navier-Stokes flux (Sec. 3.3, eq. navier-stokes-basic, read with the
    Stokes bulk term -2/3 (div v) I): a longitudinal wave v_x = A sin 2 pi x
    (rho = P = 1) has the viscous momentum RHS (4/3) nu d2v_x/dx2 and the
    viscous energy RHS d/dx(v_x Pi_xx) = (16/3) pi^2 nu A^2 cos 4 pi x; a
    transverse wave v_y = A sin 2 pi x has the energy RHS
    d/dx(v_y Pi_yx) = 4 pi^2 nu A^2 cos 4 pi x.  L(nu) - L(0) removes every
    inviscid term, and the remainder converges to these values with the
    mesh.  Dropping the bulk term changes 4/3 to 2, dropping v.Pi removes the
    energy term: both fail here.
  * HLLC star states (Toro, ch. 10): for subsonic data, the intermediate state
    U*_K recovered from F = F_K + S_K (U*_K - U_K) (Rankine-Hugoniot across
    the outer wave) moves with the contact speed S*, keeps the tangential
    velocity, and F is the flux of U*_K with the common star pressure
    p* = p_K + rho_K (S_K - u_K)(S* - u_K) (the same from both sides):
    F = (rho* S*, rho* S* v* + p* e_n, S* (E* + p*)), i.e. Rankine-Hugoniot
    across the contact.  (The star pressure is not the equation-of-state
    pressure of U*_K; the scheme defines it by these relations.)
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2208_11131_amd import workloads as W


# --------------------------------------------------------------------------
# driving source
# --------------------------------------------------------------------------

def _poly_state(prob, rng, v, P=1.0):
    """rho: random polynomial of degree <= n per axis around 1 (exactly
    representable); uniform velocity v and pressure P."""
    d, g = prob.dim, prob.p.gamma
    M = prob.nmodes
    w = np.zeros(prob.shape)
    rho = np.zeros((prob.ncells, M))
    rho[:, 0] = 1.0 + 0.2 * rng.random(prob.ncells)
    rho[:, 1:] = 0.02 * rng.standard_normal((prob.ncells, M - 1))
    w[:, 0] = rho
    for i in range(d):
        w[:, 1 + i] = v[i] * rho
    # E = P/(g-1) + 1/2 rho |v|^2 is again a polynomial of the same degree
    w[:, d + 1] = 0.5 * sum(vi * vi for vi in v[:d]) * rho
    w[:, d + 1, 0] += P / (g - 1.0)
    return w


@pytest.mark.parametrize("order", [2, 3])
def test_forcing_source_uniform_acceleration(order):
    """Uniform acceleration s: d(rho v)/dt gains s_i w_rho, dE/dt gains
    (s.v) w_rho, the density is untouched (all modes, exact)."""
    n = (3, 2, 2)
    rng = np.random.default_rng(order)
    prob = O.Problem(3, n, 0.2, order, 1.4)
    v = (0.3, -0.2, 0.5)
    w = _poly_state(prob, rng, v)
    s = np.array([0.7, -1.1, 0.4])
    sc = np.zeros((prob.ncells, 3, prob.nmodes))
    sc[:, :, 0] = s
    L0 = prob.rhs(w)
    prob.set_forcing(sc)
    L1 = prob.rhs(w)
    dL = L1 - L0
    rho = w[:, 0]
    scale = np.abs(rho).max()
    np.testing.assert_allclose(dL[:, 0], 0.0, atol=1e-14 * scale)
    for i in range(3):
        np.testing.assert_allclose(dL[:, 1 + i], s[i] * rho, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(dL[:, 4], float(s @ np.array(v)) * rho, rtol=0, atol=1e-13 * scale)


def test_forcing_source_linear_acceleration_uniform_gas():
    """rho = 1.7, v uniform, s_x = a + b Pt_1(xi_x) in every cell: the
    momentum RHS gains rho (a, b) in modes (0, l_x = 1), the energy rho v_x (a, b)."""
    order = 3
    prob = O.Problem(3, (2, 2, 2), 0.25, order, 1.4)
    v = (0.4, 0.1, -0.3)
    rho0 = 1.7
    w = np.zeros(prob.shape)
    w[:, 0, 0] = rho0
    for i in range(3):
        w[:, 1 + i, 0] = rho0 * v[i]
    w[:, 4, 0] = 1.0 / 0.4 + 0.5 * rho0 * sum(x * x for x in v)
    a, b = 0.9, -0.35
    sc = np.zeros((prob.ncells, 3, prob.nmodes))
    sc[:, 0, 0] = a
    sc[:, 0, 1] = b                      # mode l = (1, 0, 0)
    L0 = prob.rhs(w)
    prob.set_forcing(sc)
    dL = prob.rhs(w) - L0
    exp_m = np.zeros(prob.nmodes)
    exp_m[0], exp_m[1] = rho0 * a, rho0 * b
    np.testing.assert_allclose(dL[:, 1], np.broadcast_to(exp_m, (prob.ncells, prob.nmodes)), rtol=0, atol=1e-13)
    np.testing.assert_allclose(dL[:, 2:4], 0.0, atol=1e-13)
    np.testing.assert_allclose(dL[:, 4], np.broadcast_to(v[0] * exp_m, (prob.ncells, prob.nmodes)), rtol=0,
                               atol=1e-13)
    np.testing.assert_allclose(dL[:, 0], 0.0, atol=1e-13)


# --------------------------------------------------------------------------
# Navier-Stokes momentum (bulk term) and energy (v.Pi) rows
# --------------------------------------------------------------------------

def _viscous_part(order, n, comp, nu=1e-2, A=0.05):
    """L(nu) - L(0) for rho = P = 1 and v_comp = A sin 2 pi x on an n x n
    periodic grid, with the projected exact viscous RHS."""
    g = 1.4

    def fn(X):
        x, y = X
        s = A * torch.sin(2 * math.pi * x)
        z = torch.zeros_like(x)
        vel = [s, z] if comp == 0 else [z, s]
        return W._conserved(torch.ones_like(x), vel, torch.ones_like(x), g)

    h = 1.0 / n
    w = W.project(fn, 2, (n, n), (0.0, 0.0), h, order).numpy()
    visc = O.Problem(2, (n, n), h, order, g, nu=nu)
    invisc = O.Problem(2, (n, n), h, order, g)
    dL = visc.rhs(w) - invisc.rhs(w)
    k2 = 4 * math.pi ** 2
    mom_c = (4.0 / 3.0) if comp == 0 else 1.0          # Pi_xx = 4/3 nu rho v_x' ; Pi_yx = nu rho v_y'

    def ex(X):
        x, y = X
        z = torch.zeros_like(x)
        m = -mom_c * nu * k2 * A * torch.sin(2 * math.pi * x)
        # d/dx (v Pi) = mom_c nu d/dx (v v') = mom_c nu (1/2) d2/dx2 (A sin)^2 = mom_c nu A^2 4 pi^2 cos 4 pi x
        e = mom_c * nu * A * A * 4 * math.pi ** 2 * torch.cos(4 * math.pi * x)
        mom = [m, z] if comp == 0 else [z, m]
        return torch.stack([z, mom[0], mom[1], e])

    E = W.project(ex, 2, (n, n), (0.0, 0.0), h, order).numpy()
    mscale = mom_c * nu * k2 * A
    escale = mom_c * nu * A * A * 4 * math.pi ** 2
    em = np.abs(dL[:, 1 + comp, 0] - E[:, 1 + comp, 0]).max() / mscale
    ee = np.abs(dL[:, 3, 0] - E[:, 3, 0]).max() / escale
    eo = np.abs(dL[:, 2 - comp]).max() / mscale       # the other momentum component stays 0
    return em, ee, eo


@pytest.mark.parametrize("comp", [0, 1])
def test_viscous_rows_by_value(comp):
    """Cell means of the viscous momentum and energy RHS converge to the exact
    values at second order or better (p = 3), within 2 % at 32 cells."""
    errs = [_viscous_part(3, n, comp) for n in (8, 16, 32)]
    em = [e[0] for e in errs]
    ee = [e[1] for e in errs]
    assert em[-1] < 0.02 and ee[-1] < 0.02, errs
    assert math.log2(em[-2] / em[-1]) > 1.8 and math.log2(ee[-2] / ee[-1]) > 1.8, errs
    assert max(e[2] for e in errs) < 1e-10, errs


def test_bulk_term_coefficient():
    """The longitudinal wave's viscous momentum cell means approach 4/3 nu
    v_x'' and not 2 nu v_x'' (no bulk term) or 2/3 nu v_x'' (+2/3 bulk term,
    read literally with the opposite sign): the relative error at 32 cells is
    far below the 1/3 gap between these readings."""
    em, _, _ = _viscous_part(4, 32, 0)
    assert em < 0.01


# --------------------------------------------------------------------------
# HLLC star states
# --------------------------------------------------------------------------

def _cons(rho, v, p, g):
    v = np.asarray(v, dtype=float)
    return np.array([rho, *(rho * v), p / (g - 1.0) + 0.5 * rho * (v @ v)])


@pytest.mark.parametrize("dim", [2, 3])
def test_hllc_star_state_rankine_hugoniot(dim):
    g = 1.4
    rng = np.random.default_rng(17 + dim)
    n_left = n_right = 0
    for trial in range(200):
        rl, rr = rng.uniform(0.3, 2.0, 2)
        pl, pr = rng.uniform(0.3, 2.0, 2)
        vl = rng.uniform(-0.4, 0.4, dim)
        vr = rng.uniform(-0.4, 0.4, dim)
        uL, uR = _cons(rl, vl, pl, g), _cons(rr, vr, pr, g)
        a = int(rng.integers(0, dim))
        F = O.hllc(dim, g, uL, uR, a)
        cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
        SL = min(vl[a] - cl, vr[a] - cr)
        SR = max(vl[a] + cl, vr[a] + cr)
        assert SL < 0 < SR                                        # subsonic data: a star branch
        Ss = (pr - pl + rl * vl[a] * (SL - vl[a]) - rr * vr[a] * (SR - vr[a])) / (rl * (SL - vl[a]) - rr * (SR - vr[a]))
        if Ss >= 0:
            uK, S, rK, vK, pK = uL, SL, rl, vl, pl
            n_left += 1
        else:
            uK, S, rK, vK, pK = uR, SR, rr, vr, pr
            n_right += 1
        us = uK + (F - O.euler_flux(dim, g, uK, a)) / S                # RH across the outer wave
        rs = us[0]
        vs = us[1:1 + dim] / rs
        pstar = pK + rK * (S - vK[a]) * (Ss - vK[a])
        assert abs(vs[a] - Ss) <= 1e-12 * (1 + abs(Ss)), (trial, vs[a], Ss)
        # the other branch's star pressure is the same (contact: no pressure jump)
        pother = (pl + rl * (SL - vl[a]) * (Ss - vl[a])) if Ss < 0 else (pr + rr * (SR - vr[a]) * (Ss - vr[a]))
        assert abs(pother - pstar) <= 1e-12 * pstar
        tang = [i for i in range(dim) if i != a]
        np.testing.assert_allclose(vs[tang], vK[tang], rtol=1e-12, atol=1e-14)
        Fc = np.concatenate([[rs * Ss], rs * Ss * vs + pstar * (np.arange(dim) == a), [Ss * (us[dim + 1] + pstar)]])
        np.testing.assert_allclose(Fc, F, rtol=1e-11, atol=1e-12)
    assert n_left > 20 and n_right > 20


# --------------------------------------------------------------------------
# the rounding scale used by the parity measures
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,nu,av", [(2, 3e-3, {}), (3, 3e-3, None)])
def test_rounding_scale_bounds_the_rhs(dim, nu, av):
    """The per-coefficient sum of summand magnitudes bounds |L| (triangle
    inequality) and is positive wherever any summand is; on a free stream,
    where L = 0 exactly, it keeps the scale of the flux sums."""
    n = (4, 3, 2)[:dim]
    prob = O.Problem(dim, n, 0.25, 3, 1.4, nu=nu, kappa=nu, av=av)
    w = W.random_smooth(dim, n, 3, nfields=prob.nfields, seed=5, amp=0.1,
                        alpha_level=0.3 if av is not None else 0.0).numpy()
    R = np.zeros(prob.ncells) if av is not None else None
    L = prob.rhs(w, R_prev=R)
    S = prob.rhs_abs(w, R_prev=R)
    assert np.all(S >= np.abs(L) * (1 - 1e-14))
    cells = np.array([0, prob.ncells - 1])
    np.testing.assert_array_equal(prob.rhs_abs(w, cells=cells, R_prev=R), S[cells])
    wu = np.zeros_like(w)
    wu[:, 0, 0] = 1.0
    wu[:, 1, 0] = 0.5
    wu[:, dim + 1, 0] = 2.0
    Lu = prob.rhs(wu, R_prev=R)
    Su = prob.rhs_abs(wu, R_prev=R)
    assert Su[:, dim + 1].max() > 1.0 and np.abs(Lu).max() < 1e-13 * Su.max()
