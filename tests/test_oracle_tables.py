"""Oracle pins: basis, quadrature, mode counts, RK stage counts.

Each check compares the oracle with something other than itself: numpy's
Gauss-Legendre and Legendre routines (library special cases), closed forms of
the scaled Legendre basis (Sec. 2.3), and the memory table the paper prints
(Sec. 8.3, Table tab:mem), which fixes both the mode count of the paper's
total-degree basis and the RK stage count f_t(p).
"""
import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", range(1, 11))
def test_gauss_matches_numpy(n):
    x, w = O.gauss(n)
    xn, wn = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xn, atol=2e-15)
    np.testing.assert_allclose(w, wn, atol=2e-15)


@pytest.mark.parametrize("n", range(1, 11))
def test_gauss_exact_to_degree_2n_minus_1(n):
    x, w = O.gauss(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((w * x ** k).sum() - exact) < 1e-14
    # and not exact at degree 2n (the rule has exactly n points)
    k = 2 * n
    assert abs((w * x ** k).sum() - 2.0 / (k + 1)) > 1e-6


def test_legendre_values_match_numpy():
    rng = np.random.default_rng(1)
    for x in list(rng.uniform(-1, 1, 7)) + [-1.0, 0.0, 1.0]:
        P, dP = O.legendre(9, x)
        for l in range(10):
            c = np.zeros(l + 1)
            c[l] = 1.0
            ref = math.sqrt(2 * l + 1) * np.polynomial.legendre.legval(x, c)
            dref = math.sqrt(2 * l + 1) * np.polynomial.legendre.legval(x, np.polynomial.legendre.legder(c))
            assert abs(P[l] - ref) < 1e-13
            assert abs(dP[l] - dref) < 1e-11 * max(1, abs(dref))


def test_legendre_endpoints_closed_form():
    # Pt_l(+-1) = (+-1)^l sqrt(2l+1)
    P1, _ = O.legendre(9, 1.0)
    Pm, _ = O.legendre(9, -1.0)
    for l in range(10):
        assert abs(P1[l] - math.sqrt(2 * l + 1)) < 1e-13
        assert abs(Pm[l] - (-1) ** l * math.sqrt(2 * l + 1)) < 1e-13


def test_orthonormal_basis():
    # (1/2) int Pt_l Pt_m = delta_lm  (Sec. 2.3 normalisation)
    x, w = O.gauss(12)
    V = np.array([O.legendre(9, xi)[0] for xi in x])
    G = 0.5 * (V * w[:, None]).T @ V
    np.testing.assert_allclose(G, np.eye(10), atol=1e-13)


def _n3d(n):
    return (n + 1) * (n + 2) * (n + 3) // 6


def test_total_degree_mode_counts():
    # eq. N3D / N2D against enumeration
    for n in range(10):
        cnt3 = sum(1 for a in range(n + 1) for b in range(n + 1) for c in range(n + 1) if a + b + c <= n)
        cnt2 = sum(1 for a in range(n + 1) for b in range(n + 1) if a + b <= n)
        assert cnt3 == _n3d(n)
        assert cnt2 == (n + 1) * (n + 2) // 2


def test_memory_table_pins_stage_count():
    """The printed memory table equals [3+d+f_t(order)] N_c^3 N3D(n) * 8 B with
    f_t from the oracle's RK stage count: pins f_t(p) = p for p <= 3, 5 beyond."""
    unit = {"MB": 2.0 ** 20, "GB": 2.0 ** 30, "TB": 2.0 ** 40}
    rows = 0
    with open(os.path.join(GOLDEN, "memory_table.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            nc, deg, val, u = line.split()
            nc, deg, val = int(nc), int(deg), float(val)
            ft = O.rk_stages(deg + 1)
            need = (3 + 3 + ft) * nc ** 3 * _n3d(deg) * 8.0 / unit[u]
            # printed to 3-4 significant digits
            assert abs(need - val) / val < 2e-3, (nc, deg, need, val)
            rows += 1
    assert rows == 10


def test_stage_counts():
    assert [O.rk_stages(p) for p in range(1, 9)] == [1, 2, 3, 5, 5, 5, 5, 5]


def test_recovery_fraction():
    # f = 3/4 for n <= 2, f = 1 for n > 2 (Sec. 3.2); n = p - 1
    assert [O.recovery_fraction(p) for p in range(1, 9)] == [0.75] * 3 + [1.0] * 5
