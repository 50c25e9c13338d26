"""Error measures used to compare GPU results with the oracle (test
infrastructure).

Fields are compared in physical groups: density, the momentum vector (all
components together, so an identically-zero component is measured against the
momentum scale), total energy, and the AV field alpha.

  rhs_err(L, Lr, S)  max_g ||L_g - Lr_g||_inf / ||S_g||_inf, where S is the
                     oracle's rounding scale of the RHS (Problem.rhs_abs: per
                     coefficient, the sum of the magnitudes of the summands of
                     its volume, source and surface sums).  Two correct
                     evaluations of the same quadrature sums in a different
                     order (sum factorisation, other point-value paths) differ
                     by a modest multiple of the unit roundoff times S, so a
                     bound of 1e-12 leaves room for the accumulated rounding of
                     some hundred operations and nothing more.
  rhs_plain(L, Lr)   max_g ||L_g - Lr_g||_inf / ||Lr_g||_inf, recorded next to
                     it.  Where the RHS is a small difference of large
                     summands (a shear layer near equilibrium, the energy
                     equation at gamma -> 1) this plain ratio is bounded by
                     the rounding of the summands, u S / ||L||, not by u.
  state_err(a, b)    max_g ||a_g - b_g||_inf / max(||b_g||_inf, floor_g)
                     The momentum group's magnitude is at least
                     ||rho||_inf (c_max + v_max) (mom_scale), so that a flow
                     at rest is not measured against a zero norm.
  incr_err(a, b, w0) the same groups for the increments a - w0 and b - w0 of
                     one or more steps from w0 (relative to the oracle's
                     increment): what a step adds is measured on its own scale.
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


def incr_err(a, b, w0, dim):
    """Group-wise ||(a - w0) - (b - w0)||_inf / ||b - w0||_inf (groups whose
    oracle increment is zero are skipped)."""
    a = np.asarray(a)
    b = np.asarray(b)
    w0 = np.asarray(w0)
    e = 0.0
    for g in groups(b.shape[1], dim):
        db = b[:, g] - w0[:, g]
        den = np.abs(db).max()
        if den == 0.0:
            continue
        e = max(e, np.abs((a[:, g] - w0[:, g]) - db).max() / den)
    return e


def rhs_err(L, Lr, S, dim):
    """max_g ||L_g - Lr_g||_inf / ||S_g||_inf (S: the oracle's rounding scale)."""
    L = np.asarray(L)
    Lr = np.asarray(Lr)
    S = np.asarray(S)
    e = 0.0
    for g in groups(Lr.shape[1], dim):
        den = np.abs(S[:, g]).max()
        num = np.abs(L[:, g] - Lr[:, g]).max()
        e = max(e, num / den if den > 0 else num)
    return e


def rhs_plain(L, Lr, dim):
    """Per group ||L_g - Lr_g||_inf / ||Lr_g||_inf (a list: rho, momentum,
    energy[, alpha]); a group with Lr_g = 0 reports the absolute difference."""
    L = np.asarray(L)
    Lr = np.asarray(Lr)
    out = []
    for g in groups(Lr.shape[1], dim):
        den = np.abs(Lr[:, g]).max()
        num = np.abs(L[:, g] - Lr[:, g]).max()
        out.append(float(num / den if den > 0 else num))
    return out


def momentum_scale(prob, w):
    """||rho||_inf (c_max + v_max): the magnitude of momentum fluctuations."""
    _, cm, vm = prob.max_dt(w)
    return float(np.abs(np.asarray(w)[:, 0]).max() * (cm + vm))
