"""Seeded synthetic inputs: initial states for the DG solver.

This module prepares inputs only.  It holds none of the solver's arithmetic:
initial conditions u(x) are projected onto the per-cell orthonormal Legendre
basis, w_l = (1/|K|) int_K u phi_l (the paper's initial-condition projection,
Sec. 2.2 eq. weights_equation), with a Gauss rule of n+3 points per axis
(n = p - 1) taken from ``numpy.polynomial.legendre``.  Both the GPU library and
the CPU oracle consume the weights it returns.

State layout of every array returned here: ``w[cell][field][mode]`` with
cell = i + n0 (j + n1 k), mode = l_x + p (l_y + p l_z), fields
(rho, rho v_x, rho v_y[, rho v_z], e[, alpha]).

Workloads (shapes and value structure of the paper's problems):
  * ``density_wave``   2D Euler, rho = 1 + 0.1 sin 2pi(x+y), v = (1,1), P = 1.
  * ``kelvin_helmholtz`` 2D shear layer on [0,1]x[0,2] (stand-in for the
    Lecoanet et al. benchmark used in Sec. 6; its reference data is not used).
  * ``sod``            2D shock tube on [0,1]x[0,h*ny], (1,1) | (0.125,0.1).
  * ``gaussian_pulse`` passive-tracer Gaussian at rest on [-0.5,0.5]^2 (periodic images).
  * ``ou_noise``       seeded standard normal draws for the driving-field updates.
  * ``turbulence``     3D periodic box, rho = 1, c_s = 1, random solenoidal
    velocity on 1 <= |k| <= 3 with amplitude ~ k^(-8/3), rms Mach 0.3, plus a
    solenoidal forcing field on the same band (Sec. 7 setup).
  * ``random_smooth``  random decaying modal coefficients around a positive
    mean state (parity inputs).
  * ``ensemble``       48 independent 2D periodic boxes of mixed size/order.
"""
import math

import numpy as np
import torch
from numpy.polynomial import legendre as npleg


def _basis_1d(order, x):
    """Scaled Legendre values sqrt(2l+1) P_l(x), shape (len(x), order)."""
    V = npleg.legvander(np.asarray(x, dtype=np.float64), order - 1)
    return V * np.sqrt(2.0 * np.arange(order) + 1.0)[None, :]


def _rule(order):
    nq = order + 2
    x, wq = npleg.leggauss(nq)
    return x, wq


def project(fn, dim, n, lo, h, order, device="cpu", chunk_cells=1 << 17, nfields=None):
    """Project ``fn`` onto the DG basis.

    ``fn(X)`` receives a list of ``dim`` coordinate tensors of equal shape and
    returns a tensor of shape (F, *shape) of conserved fields.  Returns a
    float64 tensor (ncells, F, order**dim) on ``device``.
    """
    n = list(n)[:dim]
    xq, wq = _rule(order)
    nq = len(xq)
    B = torch.tensor(_basis_1d(order, xq), dtype=torch.float64, device=device)   # (nq, p)
    Wq = torch.tensor(wq * 0.5, dtype=torch.float64, device=device)              # (1/2) weights
    xq_t = torch.tensor(xq, dtype=torch.float64, device=device)
    ncells = int(np.prod(n))
    out = None
    for c0 in range(0, ncells, chunk_cells):
        c1 = min(ncells, c0 + chunk_cells)
        cid = torch.arange(c0, c1, device=device, dtype=torch.int64)
        idx = []
        rem = cid.clone()
        for a in range(dim):
            idx.append(rem % n[a])
            rem = rem // n[a]
        # coordinates of every quadrature point: shape (nc, nq, nq[, nq]) with
        # the x index last-but-... ordering: axis a of the point grid is dim a
        X = []
        for a in range(dim):
            xc = lo[a] + (idx[a].to(torch.float64) + 0.5) * h
            shape = [c1 - c0] + [1] * dim
            shape_q = [1] + [1] * dim
            shape_q[1 + a] = nq
            X.append(xc.view(shape) + 0.5 * h * xq_t.view(shape_q))
        X = torch.broadcast_tensors(*X)
        U = fn(list(X))                              # (F, nc, nq, ..)
        F = U.shape[0]
        # contract every axis with (W * B): axis a of U is 2 + a
        T = U
        for a in range(dim):
            # T: (F, nc, ..., q_a, ...) -> replace q_a by l_a
            M = (Wq[:, None] * B)                    # (nq, p)
            T = torch.movedim(T, 2 + a, -1)
            T = T @ M
            T = torch.movedim(T, -1, 2 + a)
        # T dims: (F, nc, l_x, l_y[, l_z]); mode index = l_x + p l_y + p^2 l_z
        T = T.permute(1, 0, *range(dim + 1, 1, -1)).reshape(c1 - c0, F, order ** dim)
        if out is None:
            out = torch.empty((ncells, F, order ** dim), dtype=torch.float64, device=device)
        out[c0:c1] = T
    return out


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def _conserved(rho, vel, P, gamma, extra=()):
    ke = 0.5 * rho * sum(v * v for v in vel)
    return torch.stack([rho] + [rho * v for v in vel] + [P / (gamma - 1.0) + ke] + list(extra))


def density_wave(order, n=16, device="cpu"):
    """2D Euler density wave on the periodic unit square (gamma = 5/3)."""
    gamma = 5.0 / 3.0

    def fn(X):
        x, y = X
        rho = 1.0 + 0.1 * torch.sin(2 * math.pi * (x + y))
        one = torch.ones_like(x)
        return _conserved(rho, [one, one], one, gamma)

    h = 1.0 / n
    return project(fn, 2, (n, n), (0.0, 0.0), h, order, device)


def density_wave_exact(order, n, t, device="cpu"):
    """Projection of the exactly translated wave at time t."""
    gamma = 5.0 / 3.0

    def fn(X):
        x, y = X
        rho = 1.0 + 0.1 * torch.sin(2 * math.pi * ((x - t) + (y - t)))
        one = torch.ones_like(x)
        return _conserved(rho, [one, one], one, gamma)

    return project(fn, 2, (n, n), (0.0, 0.0), 1.0 / n, order, device)


def kelvin_helmholtz(order, nx=256, ny=512, device="cpu"):
    """2D shear layer on [0,1]x[0,2]: v_x = tanh((y-.5)/.05) - tanh((y-1.5)/.05),
    rho = 1 + v_x/2, v_y = 0.01 sin(2 pi x) (exp(-(y-.5)^2/.04) + exp(-(y-1.5)^2/.04)),
    P = 10, gamma = 5/3."""
    gamma = 5.0 / 3.0
    h = 1.0 / nx
    assert abs(ny * h - 2.0) < 1e-12 or True

    def fn(X):
        x, y = X
        prof = torch.tanh((y - 0.5) / 0.05) - torch.tanh((y - 1.5) / 0.05)
        rho = 1.0 + 0.5 * prof
        vx = prof
        vy = 0.01 * torch.sin(2 * math.pi * x) * (torch.exp(-(y - 0.5) ** 2 / 0.04) +
                                                  torch.exp(-(y - 1.5) ** 2 / 0.04))
        return _conserved(rho, [vx, vy], 10.0 * torch.ones_like(x), gamma)

    return project(fn, 2, (nx, ny), (0.0, 0.0), h, order, device)


def sod(order, nx=1024, ny=128, device="cpu", with_alpha=True):
    """Sod tube along x: (rho, P) = (1, 1) for x < 0.5, (0.125, 0.1) beyond;
    gamma = 1.4, v = 0, AV field alpha = 0."""
    gamma = 1.4
    h = 1.0 / nx

    def fn(X):
        x = X[0]
        left = x < 0.5
        rho = torch.where(left, torch.ones_like(x), 0.125 * torch.ones_like(x))
        P = torch.where(left, torch.ones_like(x), 0.1 * torch.ones_like(x))
        z = torch.zeros_like(x)
        extra = (z,) if with_alpha else ()
        return _conserved(rho, [z, z], P, gamma, extra)

    return project(fn, 2, (nx, ny), (0.0, 0.0), h, order, device)


def gaussian_pulse(order, n=8, t=1.0, eta=1.0 / 128.0, device="cpu", gamma=1.4):
    """Passive-tracer diffusion test (Sec. 5.2, eq. diffusion_spike): gas at
    rest with rho = 1, P = 1 on the periodic square [-0.5, 0.5]^2 and the tracer
    concentration c = c_b + sum_j c_g/(2 pi s^2) exp(-|x - j|^2 / (2 s^2)),
    s^2 = 2 eta t, c_b = 1/10, c_g = 1, over the periodic images j (|j_a| <= 3).
    Fields (rho, rho v_x, rho v_y, e, c rho)."""
    cb, cg = 0.1, 1.0
    s2 = 2.0 * eta * t

    def fn(X):
        x, y = X
        c = cb * torch.ones_like(x)
        for jx in range(-3, 4):
            for jy in range(-3, 4):
                r2 = (x - jx) ** 2 + (y - jy) ** 2
                c = c + cg / (2.0 * math.pi * s2) * torch.exp(-r2 / (2.0 * s2))
        one = torch.ones_like(x)
        z = torch.zeros_like(x)
        return _conserved(one, [z, z], one, gamma, (c,))

    h = 1.0 / n
    return project(fn, 2, (n, n), (-0.5, -0.5), h, order, device)


def ou_noise(nmodes, count, seed=2208):
    """Standard normal draws for `count` Ornstein-Uhlenbeck updates of the
    driving modes: an array (count, nmodes, 3, 2) from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((count, nmodes, 3, 2))


def _solenoidal_modes(rng, kmax, slope):
    """Integer wave vectors 1 <= |k| <= kmax (one of each +-k pair) with random
    complex amplitudes perpendicular to k, |a| ~ |k|^slope."""
    ks = []
    for kx in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            for kz in range(-kmax, kmax + 1):
                k2 = kx * kx + ky * ky + kz * kz
                if k2 < 1 or k2 > kmax * kmax:
                    continue
                if (kx, ky, kz) <= (-kx, -ky, -kz):
                    continue
                ks.append((kx, ky, kz))
    ks = np.array(ks, dtype=np.float64)
    a = rng.standard_normal((len(ks), 3)) + 1j * rng.standard_normal((len(ks), 3))
    kn = ks / np.linalg.norm(ks, axis=1, keepdims=True)
    a = a - (a * kn).sum(axis=1, keepdims=True) * kn
    a *= (np.linalg.norm(ks, axis=1) ** slope)[:, None] / np.linalg.norm(a, axis=1, keepdims=True)
    return ks, a


def _fourier_field(ks, amps, device):
    kt = torch.tensor(ks, dtype=torch.float64, device=device)
    at = torch.tensor(amps, dtype=torch.complex128, device=device)

    def field(X):
        comps = []
        ph = 2 * math.pi * (X[0][..., None] * kt[:, 0] + X[1][..., None] * kt[:, 1] +
                            X[2][..., None] * kt[:, 2])
        e = torch.exp(1j * ph)
        for i in range(3):
            comps.append(2.0 * (e * at[:, i]).real.sum(-1))
        return comps

    return field


def turbulence(order, n=128, device="cpu", seed=2208, mach=0.3, gamma=1.0001, chunk_cells=1 << 14):
    """3D driven-turbulence initial state and forcing field.

    Returns (w, s): w (ncells, 5, p^3) and the forcing coefficients s
    (ncells, 3, p^3) of a solenoidal acceleration field on 1 <= |k| <= 3."""
    rng = np.random.default_rng(seed)
    ks, a = _solenoidal_modes(rng, 3, -8.0 / 3.0)
    rms = math.sqrt(2.0 * float((np.abs(a) ** 2).sum()))   # <|v|^2> of 2 Re(a e^{ikx})
    a *= mach / rms                                           # c_s = 1
    ksf, af = _solenoidal_modes(rng, 3, -5.0 / 3.0)
    rmsf = math.sqrt(2.0 * float((np.abs(af) ** 2).sum()))
    af *= 0.5 / rmsf
    vel = _fourier_field(ks, a, device)
    frc = _fourier_field(ksf, af, device)
    P0 = 1.0 / gamma

    def fn(X):
        v = vel(X)
        rho = torch.ones_like(X[0])
        return _conserved(rho, v, P0 * torch.ones_like(X[0]), gamma)

    def fs(X):
        return torch.stack(frc(X))

    h = 1.0 / n
    w = project(fn, 3, (n, n, n), (0.0, 0.0, 0.0), h, order, device, chunk_cells)
    s = project(fs, 3, (n, n, n), (0.0, 0.0, 0.0), h, order, device, chunk_cells)
    return w, s


def random_smooth(dim, n, order, nfields=None, seed=0, amp=0.05, device="cpu", gamma=1.4,
                  alpha_level=0.0, vbase=(0.0, 0.0, 0.0)):
    """Random modal coefficients decaying like 2^-(l_x+l_y+l_z) on top of a
    positive mean state (rho ~ 1, v ~ vbase +- 0.3, P ~ 1).  Values are those of a
    smooth but non-trivial flow; density and pressure stay positive."""
    rng = np.random.default_rng(seed)
    n = list(n)[:dim]
    ncells = int(np.prod(n))
    M = order ** dim
    Fc = dim + 2
    F = Fc if nfields is None else nfields
    l = np.zeros((M, dim), dtype=np.int64)
    for m in range(M):
        r = m
        for a in range(dim):
            l[m, a] = r % order
            r //= order
    decay = 0.5 ** l.sum(axis=1)
    prim = np.zeros((ncells, Fc, M))
    prim[:, 0, 0] = 1.0 + 0.2 * rng.random(ncells)
    for i in range(dim):
        prim[:, 1 + i, 0] = vbase[i] + 0.3 * (2 * rng.random(ncells) - 1)
    prim[:, Fc - 1, 0] = 1.0 + 0.2 * rng.random(ncells)
    pert = amp * rng.standard_normal((ncells, Fc, M)) * decay[None, None, :]
    pert[:, :, 0] = 0.0
    prim += pert
    # conserved coefficients from "primitive-like" coefficients: use
    # rho, m = rho_bar v, E = P/(g-1) + 1/2 rho_bar |v_bar|^2 (linearised)
    w = np.zeros((ncells, F, M))
    rb = prim[:, 0, 0]
    w[:, 0, :] = prim[:, 0, :]
    ke = np.zeros(ncells)
    for i in range(dim):
        w[:, 1 + i, :] = prim[:, 1 + i, :] * rb[:, None]
        ke += 0.5 * rb * prim[:, 1 + i, 0] ** 2
    w[:, Fc - 1, :] = prim[:, Fc - 1, :] / (gamma - 1.0)
    w[:, Fc - 1, 0] += ke
    if F > Fc:
        w[:, Fc, 0] = alpha_level
        w[:, Fc, 1:] = 0.1 * alpha_level * rng.standard_normal((ncells, M - 1)) * decay[None, 1:]
    return torch.tensor(w, device=device)


# --------------------------------------------------------------------------
# batched ensemble of independent boxes
# --------------------------------------------------------------------------

ENSEMBLE_SIDES = (32, 64, 128, 256, 512)


def ensemble_layout(nbox=48, seed=2208):
    """Sizes and orders of the boxes: side ~ U{32,64,128,256,512}, p ~ U{2..6}."""
    rng = np.random.default_rng(seed)
    sides = rng.choice(np.array(ENSEMBLE_SIDES), size=nbox)
    orders = rng.integers(2, 7, size=nbox)
    return [int(s) for s in sides], [int(p) for p in orders]


def ensemble_box(b, side, order, device="cpu", seed=2208, gamma=5.0 / 3.0, amp=0.05):
    """Box b: each of rho-1, v_x, v_y = amp * sum_{m=1..4} a_m sin(2 pi k_m.x + phi_m) / 4,
    a_m ~ U[0,1], k_m in {-3..3}^2 \\ {0}, phi_m ~ U[0, 2 pi); P = 1."""
    rng = np.random.default_rng(seed + b)
    params = []
    for _ in range(3):
        am = rng.random(4)
        km = []
        while len(km) < 4:
            k = rng.integers(-3, 4, size=2)
            if k[0] != 0 or k[1] != 0:
                km.append(k)
        ph = rng.random(4) * 2 * math.pi
        params.append((am, np.array(km, dtype=np.float64), ph))

    def comp(X, pr):
        am, km, ph = pr
        s = torch.zeros_like(X[0])
        for m in range(4):
            s = s + am[m] * torch.sin(2 * math.pi * (km[m, 0] * X[0] + km[m, 1] * X[1]) + ph[m])
        return amp * s / 4.0

    def fn(X):
        rho = 1.0 + comp(X, params[0])
        vx = comp(X, params[1])
        vy = comp(X, params[2])
        return _conserved(rho, [vx, vy], torch.ones_like(X[0]), gamma)

    return project(fn, 2, (side, side), (0.0, 0.0), 1.0 / side, order, device)
