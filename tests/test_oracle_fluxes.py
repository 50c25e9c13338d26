"""Oracle pins: Euler flux and HLLC Riemann flux (Sec. 2, eq. flux_matrix; Sec. 2.2).

Pins: consistency F(u,u) = f(u); supersonic upwinding; exactness at an isolated
contact (HLLC resolves contacts exactly, Toro ch. 10); mirror symmetry; the
energy row (e + p) v with e the total energy density, checked against values
written out by hand for one state.
"""
import numpy as np
import pytest

import oracle as O


def cons(dim, rho, v, P, gamma):
    v = np.asarray(v, dtype=float)
    return np.array([rho, *(rho * v), P / (gamma - 1) + 0.5 * rho * (v @ v)])


def test_euler_flux_hand_values():
    g = 1.4
    u = cons(3, 2.0, [0.5, -1.0, 0.25], 3.0, g)
    E = 3.0 / 0.4 + 0.5 * 2.0 * (0.25 + 1.0 + 0.0625)
    f = O.euler_flux(3, g, u, 1)          # y-flux
    ref = [2.0 * -1.0, 2.0 * 0.5 * -1.0, 2.0 * 1.0 + 3.0, 2.0 * 0.25 * -1.0, (E + 3.0) * -1.0]
    np.testing.assert_allclose(f, ref, rtol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_hllc_consistency(dim):
    rng = np.random.default_rng(dim)
    for _ in range(50):
        u = cons(dim, rng.uniform(0.1, 3), rng.uniform(-2, 2, dim), rng.uniform(0.1, 3), 1.4)
        for a in range(dim):
            np.testing.assert_allclose(O.hllc(dim, 1.4, u, u, a), O.euler_flux(dim, 1.4, u, a),
                                       rtol=1e-13, atol=1e-13)


def test_hllc_supersonic_upwind():
    g = 5 / 3
    uL = cons(2, 1.0, [5.0, 0.3], 1.0, g)
    uR = cons(2, 0.5, [4.0, -0.2], 0.7, g)
    np.testing.assert_allclose(O.hllc(2, g, uL, uR, 0), O.euler_flux(2, g, uL, 0), rtol=1e-14)
    uL2 = cons(2, 1.0, [-5.0, 0.3], 1.0, g)
    uR2 = cons(2, 0.5, [-4.0, -0.2], 0.7, g)
    np.testing.assert_allclose(O.hllc(2, g, uL2, uR2, 0), O.euler_flux(2, g, uR2, 0), rtol=1e-14)


@pytest.mark.parametrize("vn", [0.7, -0.4])
def test_hllc_exact_contact(vn):
    """Density jump with equal normal velocity and pressure: the exact flux is
    the upwind Euler flux (mass flux rho_upwind v_n, momentum, energy)."""
    g = 1.4
    uL = cons(3, 1.0, [vn, 0.2, -0.1], 1.0, g)
    uR = cons(3, 0.25, [vn, -0.5, 0.3], 1.0, g)
    F = O.hllc(3, g, uL, uR, 0)
    up = uL if vn > 0 else uR
    np.testing.assert_allclose(F, O.euler_flux(3, g, up, 0), rtol=1e-13, atol=1e-14)


def test_hllc_mirror_symmetry():
    """Reflecting x -> -x swaps the states and flips the normal velocity; the
    flux components then transform as (-F_rho, F_mx, -F_my, -F_E)."""
    g = 1.4
    rng = np.random.default_rng(5)
    for _ in range(30):
        uL = cons(2, rng.uniform(0.2, 2), rng.uniform(-1, 1, 2), rng.uniform(0.2, 2), g)
        uR = cons(2, rng.uniform(0.2, 2), rng.uniform(-1, 1, 2), rng.uniform(0.2, 2), g)
        F = O.hllc(2, g, uL, uR, 0)
        mL = uR * np.array([1, -1, 1, 1])
        mR = uL * np.array([1, -1, 1, 1])
        Fm = O.hllc(2, g, mL, mR, 0)
        np.testing.assert_allclose(Fm, F * np.array([-1, 1, -1, -1]), rtol=1e-12, atol=1e-13)


def test_hllc_axis_permutation():
    g = 1.4
    rng = np.random.default_rng(9)
    uL = cons(3, 1.3, rng.uniform(-1, 1, 3), 0.8, g)
    uR = cons(3, 0.6, rng.uniform(-1, 1, 3), 1.7, g)
    Fx = O.hllc(3, g, uL, uR, 0)
    perm = [0, 2, 1, 3, 4]            # swap x <-> y components
    Fy = O.hllc(3, g, uL[perm], uR[perm], 1)
    np.testing.assert_allclose(Fy[perm], Fx, rtol=1e-14, atol=1e-15)
