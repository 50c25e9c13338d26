"""GPU parity of the positivity limiter (Sec. 4.2) against the oracle.

  * dg_limit on states whose cells dip below the density / pressure bottoms
    (2D and 3D, with and without the AV field): the same cells change, and
    the limited states agree to 1e-12 per field group; a state that needs
    nothing is left bitwise unchanged;
  * SSP-RK steps with the limiter on every stage state (the option of
    dg_init), starting from a limited initial state: a strong two-state tube
    at p = 6 (the jump inside a cell) on a strip and on a 3-row box, and a 3D
    p = 4 box with dips, against the oracle's limited steps.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle.compare import momentum_scale, state_err
from paper_2208_11131_amd import workloads as W

pytestmark = pytest.mark.gpu

dg = pytest.importorskip("paper_2208_11131_amd")

G = 1.4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dipped_state(dim, n, order, F, seed, frac=0.3):
    """Random smooth state whose selected cells get large higher modes in
    density and energy (dips below zero at some limiter points)."""
    w = W.random_smooth(dim, n, order, nfields=F, seed=seed, amp=0.05,
                        alpha_level=0.2 if F > dim + 2 else 0.0).numpy()
    rng = np.random.default_rng(seed + 100)
    nc, M = w.shape[0], order ** dim
    sel = rng.random(nc) < frac
    for f, amp in ((0, 0.5), (dim + 1, 1.2)):
        w[sel, f, 1:] += amp * w[sel, f, :1] * rng.standard_normal((int(sel.sum()), M - 1))
    return np.ascontiguousarray(w)


def changed_cells(a, b):
    return np.nonzero(np.any(a != b, axis=(1, 2)))[0]


@pytest.mark.parametrize("dim,n,order,av", [(2, (13, 9), 4, False), (2, (11, 7), 6, True), (3, (4, 3, 3), 3, False),
                                            (3, (3, 3, 2), 4, True), (2, (9, 5), 8, False)])
def test_limit_matches_oracle(dim, n, order, av):
    say("limit", dim, n, order, av)
    avd = {} if av else None
    F = dim + 2 + (1 if av else 0)
    ref = O.Problem(dim, n, 1.0 / n[0], order, G, av=avd)
    gpu = dg.Solver(dim, n, order, G, av=avd)
    w0 = dipped_state(dim, n, order, F, seed=order + 10 * dim)
    wr, nchg = ref.limit(w0)
    assert nchg >= 3
    w = torch.tensor(w0, device="cuda")
    gpu.limit(w)
    wg = w.cpu().numpy()
    cg, cr = changed_cells(wg, w0), changed_cells(wr, w0)
    say("  cells changed: gpu %d, oracle %d of %d" % (len(cg), len(cr), w0.shape[0]))
    np.testing.assert_array_equal(cg, cr)
    np.testing.assert_array_equal(wg[:, :, 0], w0[:, :, 0])          # means untouched
    e = state_err(wg, wr, dim, mom_scale=momentum_scale(ref, wr))
    say("  state err %.2e" % e)
    assert e <= 1e-12


def test_limit_leaves_good_states_alone():
    dim, n, order = 2, (10, 6), 5
    gpu = dg.Solver(dim, n, order, G)
    w0 = W.random_smooth(dim, n, order, seed=4, amp=0.05).numpy()
    w = torch.tensor(w0, device="cuda")
    gpu.limit(w)
    assert torch.equal(w.cpu(), torch.tensor(w0))


def _tube(order, nx, ny):
    """Two-state tube along x (rho 1 : 1e-3, P 1 : 1e-5), the jump inside cell
    nx/2 at a third of its width (projected exactly), y-uniform."""
    M = order * order
    w = np.zeros((nx, 4, M))
    left = np.arange(nx) < nx // 2
    w[:, 0, 0] = np.where(left, 1.0, 1e-3)
    w[:, 3, 0] = np.where(left, 1.0, 1e-5) / (G - 1)
    c, x0 = nx // 2, -1.0 / 3.0
    w[c] = 0.0
    xq, wq = np.polynomial.legendre.leggauss(40)
    for lo, hi, v in ((-1.0, x0, (1.0, 1.0 / (G - 1))), (x0, 1.0, (1e-3, 1e-5 / (G - 1)))):
        x = 0.5 * (hi - lo) * xq + 0.5 * (hi + lo)
        wt = 0.5 * (hi - lo) * wq
        P = np.polynomial.legendre.legvander(x, order - 1) * np.sqrt(2 * np.arange(order) + 1)
        w[c, 0, :order] += 0.5 * v[0] * (wt[:, None] * P).sum(axis=0)
        w[c, 3, :order] += 0.5 * v[1] * (wt[:, None] * P).sum(axis=0)
    return np.ascontiguousarray(np.tile(w, (ny, 1, 1)))


@pytest.mark.parametrize("ny", [1, 3])
def test_limited_steps_strong_tube(ny):
    order, nx = 6, 24
    say("limited steps tube", ny)
    h = 1.0 / nx
    ref = O.Problem(2, (nx, ny), h, order, G, bc=(2, 0), cfl=0.3, limiter=True)
    gpu = dg.Solver(2, (nx, ny), order, G, hi=[1.0, ny * h], bc=[2, 0], cfl=0.3, limiter=True)
    w0 = _tube(order, nx, ny)
    wr, nchg = ref.limit(w0)
    assert nchg >= 1
    w = torch.tensor(w0, device="cuda")
    gpu.limit(w)
    wr0 = wr.copy()
    for _ in range(6):
        dt = ref.max_dt(wr)[0]
        assert abs(gpu.max_dt(w)[0] - dt) <= 1e-13 * dt
        gpu.step(w, dt)
        wr, _ = ref.step(wr, dt)
    assert gpu.check() == 0
    wg = w.cpu().numpy()
    e = state_err(wg, wr, 2, mom_scale=momentum_scale(ref, wr))
    say("  state err after 6 limited steps %.2e" % e)
    assert e <= 1e-12
    # the unlimited scheme does not survive the first step from this state
    off = O.Problem(2, (nx, ny), h, order, G, bc=(2, 0), cfl=0.3)
    wb, _ = off.step(wr0, ref.max_dt(wr0)[0])
    assert not np.isfinite(wb).all() or (wb[:, 0, 0] <= 0).any()


def test_limited_steps_3d():
    dim, n, order = 3, (4, 3, 3), 4
    say("limited steps 3d")
    ref = O.Problem(dim, n, 1.0 / 4, order, G, nu=1e-3, kappa=1e-3, limiter=True)
    gpu = dg.Solver(dim, n, order, G, nu=1e-3, kappa=1e-3, limiter=True)
    w0 = dipped_state(dim, n, order, dim + 2, seed=77, frac=0.4)
    wr, _ = ref.limit(w0)
    w = torch.tensor(w0, device="cuda")
    gpu.limit(w)
    dt = 0.3 * ref.max_dt(wr)[0]
    for _ in range(3):
        gpu.step(w, dt)
        wr, _ = ref.step(wr, dt)
    assert gpu.check() == 0
    e = state_err(w.cpu().numpy(), wr, dim, mom_scale=momentum_scale(ref, wr))
    say("  state err after 3 limited steps %.2e" % e)
    assert e <= 1e-12
