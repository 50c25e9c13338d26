"""Error measures used to compare GPU results with the oracle (test
infrastructure).

Fields are compared in physical groups: density, the momentum vector (all
components together, so an identically-zero component is measured against the
momentum scale), total energy, and the AV field alpha.

  state_err(a, b)    max_g ||a_g - b_g||_inf / max(||b_g||_inf, floor_g)
  rhs_err(L, Lr, w, rate)
                     max_g ||L_g - Lr_g||_inf / max(||Lr_g||_inf, rate ||w_g||_inf)
  The momentum group's magnitude is at least ||rho||_inf (c_max + v_max)
  (mom_scale), so that a flow at rest is not measured against a zero norm.
    with rate = 2 p (c_max + v_max) / h, the inverse of the unit-CFL time
    step: an RHS error below tol * rate ||w|| changes a CFL-limited step of the
    state by less than tol relative.  This is the natural scale when the RHS
    is a small difference of large fluxes (e.g. the energy equation at
    gamma -> 1, where e ~ P/(gamma-1) >> its time derivative).
"""
import numpy as np


def groups(nfields, dim):
    g = [[0], list(range(1, 1 + dim)), [dim + 1]]
    if nfields > dim + 2:
        g.append([dim + 2])
    return g


def state_err(a, b, dim, alpha_floor=1e-2, mom_scale=0.0):
    a = np.asarray(a)
    b = np.asarray(b)
    e = 0.0
    for gi, g in enumerate(groups(b.shape[1], dim)):
        den = np.abs(b[:, g]).max()
        if gi == 1:
            den = max(den, mom_scale)
        if gi == 3:
            den = max(den, alpha_floor)
        num = np.abs(a[:, g] - b[:, g]).max()
        e = max(e, num / den if den > 0 else num)
    return e


def rhs_err(L, Lr, w, dim, rate, mom_scale=0.0):
    """w may be the whole state even when L, Lr hold a subset of cells."""
    L = np.asarray(L)
    Lr = np.asarray(Lr)
    w = np.asarray(w)
    e = 0.0
    for gi, g in enumerate(groups(Lr.shape[1], dim)):
        wn = np.abs(w[:, g]).max()
        if gi == 1:
            wn = max(wn, mom_scale)
        den = max(np.abs(Lr[:, g]).max(), rate * wn)
        num = np.abs(L[:, g] - Lr[:, g]).max()
        e = max(e, num / den if den > 0 else num)
    return e


def cfl_rate(prob, w):
    """2 p (c_max + v_max) / h of the oracle problem for state w."""
    _, cm, vm = prob.max_dt(w)
    return 2.0 * prob.order * (cm + vm) / prob.h


def momentum_scale(prob, w):
    """||rho||_inf (c_max + v_max): the magnitude of momentum fluctuations."""
    _, cm, vm = prob.max_dt(w)
    return float(np.abs(np.asarray(w)[:, 0]).max() * (cm + vm))
