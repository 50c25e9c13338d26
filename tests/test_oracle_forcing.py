"""Oracle pins of the driving field (Sec. 7.1): Ornstein-Uhlenbeck mode
amplitudes on the band 1 <= |k| <= k_max with a k^(-5/3) spectrum, made
solenoidal, and their projection on the DG basis.

  * the mode set: one of each +-k pair of integer vectors in the band
    (61 in 3D and 14 in 2D for k_max = 3), in the stated order;
  * OU update: without noise the amplitudes decay by exp(-dt/t_corr) exactly,
    two half steps equal one full step; every update leaves k . a = 0; over a
    long seeded run each mode's component variance approaches the stationary
    sigma_k^2 (1 - k_c^2/|k|^2), sigma_k = sigma0 |k|^(-5/3);
  * projection: the cell means equal the exact cell averages of the Fourier
    series (products of sin(pi k_a h)/(pi k_a h)); a single mode's higher
    coefficients follow the closed form (1/2) int e^{i z xi} Pt_l(xi) dxi =
    sqrt(2l+1) i^l j_l(z) (scipy's spherical Bessel functions).
"""
import math

import numpy as np
import pytest
from scipy.special import spherical_jn

import oracle as O


def test_mode_set():
    for dim, count in ((3, 61), (2, 14)):
        kv = O.forcing_modes(dim, 3)
        assert len(kv) == count
        pts = set()
        for k in kv:
            k2 = int((k ** 2).sum())
            assert 1 <= k2 <= 9
            nz = [c for c in k if c != 0]
            assert nz[0] > 0
            assert dim == 3 or k[2] == 0
            pts.add(tuple(k))
            pts.add(tuple(-k))
        # every lattice vector of the band appears exactly once as +-k
        full = {(x, y, z) for x in range(-3, 4) for y in range(-3, 4) for z in (range(-3, 4) if dim == 3 else [0])
                if 1 <= x * x + y * y + z * z <= 9}
        assert pts == full
        assert [tuple(k) for k in kv] == sorted(tuple(k) for k in kv)


def _start(dim, seed=0):
    kv = O.forcing_modes(dim, 3)
    rng = np.random.default_rng(seed)
    a = O.ou_update(dim, kv, np.zeros((len(kv), 3, 2)), rng.standard_normal((len(kv), 3, 2)), math.inf, 1.0, 0.7)
    return kv, a


@pytest.mark.parametrize("dim", [2, 3])
def test_ou_decay_and_composition(dim):
    kv, a = _start(dim)
    z = np.zeros_like(a)
    a1 = O.ou_update(dim, kv, a, z, 0.3, 1.0, 0.7)
    np.testing.assert_allclose(a1, math.exp(-0.3) * a, rtol=1e-15, atol=1e-16 * np.abs(a).max())
    a2 = O.ou_update(dim, kv, O.ou_update(dim, kv, a, z, 0.15, 1.0, 0.7), z, 0.15, 1.0, 0.7)
    np.testing.assert_allclose(a2, a1, rtol=1e-14, atol=1e-16 * np.abs(a).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_ou_solenoidal_and_stationary_variance(dim):
    kv, a = _start(dim, seed=1)
    rng = np.random.default_rng(5)
    samples = []
    for it in range(4000):
        a = O.ou_update(dim, kv, a, rng.standard_normal(a.shape), 0.5, 1.0, 0.7)
        kd = (kv[:, :, None] * a).sum(axis=1)              # (nm, 2): k . a, re and im
        assert np.abs(kd).max() <= 1e-14
        samples.append(a.copy())
    S = np.array(samples)                                   # (T, nm, 3, 2)
    k2 = (kv ** 2).sum(axis=1).astype(float)
    sig2 = 0.7 ** 2 * k2 ** (-5.0 / 3.0)
    # per component: half the variance in each of re / im; the projection
    # removes the share k_c^2 / |k|^2
    want = 0.5 * sig2[:, None] * (1.0 - kv[:, :dim] ** 2 / k2[:, None])
    got = S[:, :, :dim, :].var(axis=(0, 3))
    rel = np.abs(got - want).sum() / want.sum()
    assert rel < 0.03, rel


@pytest.mark.parametrize("dim,order", [(2, 3), (3, 2)])
def test_projection_cell_means_and_bessel_modes(dim, order):
    kv, a = _start(dim, seed=2)
    n = (5, 4, 3)[:dim]
    h = 1.0 / 5
    lo = (0.1, -0.2, 0.05)[:dim]
    prob = O.Problem(dim, n, h, order, 1.4)
    s = O.forcing_project(prob, lo, kv, a)
    nn = list(n) + [1] * (3 - dim)
    for cell in range(prob.ncells):
        ijk = [cell % nn[0], (cell // nn[0]) % nn[1], cell // (nn[0] * nn[1])]
        xc = [lo[b] + (ijk[b] + 0.5) * h for b in range(dim)]
        for c in range(dim):
            mean = 0.0
            for i, k in enumerate(kv):
                ph = 2 * math.pi * sum(k[b] * xc[b] for b in range(dim))
                damp = 1.0
                for b in range(dim):
                    z = math.pi * k[b] * h
                    damp *= math.sin(z) / z if k[b] != 0 else 1.0
                mean += 2.0 * damp * (a[i, c, 0] * math.cos(ph) - a[i, c, 1] * math.sin(ph))
            assert abs(s[cell, c, 0] - mean) <= 1e-14 * max(1.0, abs(mean))
    # one mode: coefficient l of cell 0 along x = 2 Re(a e^{2 pi i k.x_c} prod_b sqrt(2l_b+1) i^l_b j_l_b(pi k_b h))
    i = 3
    one = np.zeros_like(a)
    one[i] = a[i]
    s1 = O.forcing_project(prob, lo, kv, one)
    k = kv[i]
    xc = [lo[b] + 0.5 * h for b in range(dim)]
    for m in range(order ** dim):
        l = [(m // order ** b) % order for b in range(dim)]
        fac = np.exp(2j * math.pi * sum(k[b] * xc[b] for b in range(dim)))
        for b in range(dim):
            fac *= math.sqrt(2 * l[b] + 1) * (1j ** l[b]) * spherical_jn(l[b], math.pi * k[b] * h)
        for c in range(dim):
            want = 2.0 * ((a[i, c, 0] + 1j * a[i, c, 1]) * fac).real
            assert abs(s1[0, c, m] - want) <= 1e-14 * max(1.0, np.abs(a[i]).max())
