"""GPU parity on the total-degree basis P_n (Sec. 2.3; dg_options.basis = 1)
against the oracle (Problem(basis=1)).

  * dg_rhs: Euler and Navier-Stokes, 2D p = 2..8 and 3D p = 3, 4, periodic
    and wall ends, within 1e-12 of the oracle's rounding scale; FP32 bulk
    within 1e-5;
  * ten SSP-RK steps (2D p = 4, 3D p = 3) within 1e-12 per field group, with
    the device CFL step equal to the oracle's; totals conserved to FP64
    rounding (FP64 and FP32 bulk);
  * the positivity limiter and the driving-field projection in the P_n layout.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle.compare import momentum_scale, rhs_err, rhs_plain, state_err
from paper_2208_11131_amd import workloads as W

pytestmark = pytest.mark.gpu

dg = pytest.importorskip("paper_2208_11131_amd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pn_state(dim, n, order, seed, amp=0.08):
    """A random smooth state restricted to total degree <= n, stored in the
    P_n order (the oracle's mode list)."""
    q = W.random_smooth(dim, n, order, seed=seed, amp=amp, vbase=(0.2, -0.1, 0.1)).numpy()
    degq = O.mode_degrees(order, dim, 0)
    degp = O.mode_degrees(order, dim, 1)
    idx = [int(np.nonzero((degq == d).all(axis=1))[0][0]) for d in degp]
    return np.ascontiguousarray(q[:, :, idx])


def pair(dim, n, order, nu=0.0, bc=None, precision="fp64", **kw):
    h = 1.0 / n[0]
    ref = O.Problem(dim, n, h, order, 1.4, nu=nu, kappa=nu, bc=bc, basis=1, **kw)
    gpu = dg.Solver(dim, n, order, 1.4, nu=nu, kappa=nu, hi=[n[a] * h for a in range(dim)], bc=bc,
                    precision=precision, basis=1, **kw)
    assert gpu.nmodes == ref.nmodes
    return gpu, ref


CASES = [(2, (13, 9), o, nu, None) for o in (2, 3, 4, 5, 6, 7, 8) for nu in (0.0, 3e-3)] + \
        [(2, (9, 7), 5, 3e-3, (2, 0)), (3, (5, 4, 3), 3, 3e-3, None), (3, (3, 3, 2), 4, 0.0, None),
         (3, (3, 3, 2), 4, 3e-3, (0, 0, 2))]


@pytest.mark.parametrize("dim,n,order,nu,bc", CASES)
def test_pn_rhs_parity(dim, n, order, nu, bc):
    say("pn rhs", dim, n, order, nu, bc)
    gpu, ref = pair(dim, n, order, nu=nu, bc=bc)
    w0 = pn_state(dim, n, order, seed=order + 3 * dim)
    L = gpu.rhs(torch.tensor(w0, device="cuda")).cpu().numpy()
    Lr = ref.rhs(w0)
    e = rhs_err(L, Lr, ref.rhs_abs(w0), dim)
    say("  rhs err / rounding scale %.2e, plain %s" % (e, ["%.1e" % x for x in rhs_plain(L, Lr, dim)]))
    assert e <= 1e-12


@pytest.mark.parametrize("dim,n,order", [(2, (11, 7), 4), (3, (4, 3, 3), 4)])
def test_pn_rhs_fp32_bulk(dim, n, order):
    gpu, ref = pair(dim, n, order, nu=3e-3, precision="fp32")
    w0 = pn_state(dim, n, order, seed=31)
    L = gpu.rhs(torch.tensor(w0, device="cuda")).cpu().numpy()
    e = rhs_err(L, ref.rhs(w0), ref.rhs_abs(w0), dim)
    say("  fp32 rhs err / rounding scale %.2e" % e)
    assert e <= 1e-5


@pytest.mark.parametrize("dim,n,order,nsteps", [(2, (12, 9), 4, 10), (2, (10, 8), 7, 3), (3, (4, 3, 3), 3, 10)])
def test_pn_step_parity(dim, n, order, nsteps):
    say("pn steps", dim, order, nsteps)
    gpu, ref = pair(dim, n, order, nu=3e-3)
    w0 = pn_state(dim, n, order, seed=40 + order)
    w = torch.tensor(w0, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    wr = w0
    for _ in range(nsteps):
        gpu.step_cfl(w, dt_dev)
        dtr = ref.max_dt(wr)[0]
        assert abs(float(dt_dev) - dtr) <= 1e-14 * dtr
        wr, _ = ref.step(wr, float(dt_dev))
    assert gpu.check() == 0
    e = state_err(w.cpu().numpy(), wr, dim, mom_scale=momentum_scale(ref, wr))
    say("  state err %.2e" % e)
    assert e <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pn_conservation(precision):
    dim, n, order = 3, (5, 4, 4), 4
    gpu, ref = pair(dim, n, order, nu=3e-3, precision=precision)
    w0 = pn_state(dim, n, order, seed=70)
    w = torch.tensor(w0, device="cuda")
    t0 = np.array(gpu.totals(w))
    dt = 0.5 * ref.max_dt(w0)[0]
    for _ in range(10):
        gpu.step(w, dt)
    t1 = np.array(gpu.totals(w))
    scale = np.abs(t0) + np.abs(t0).max()
    say("  drift / scale", ["%.1e" % x for x in np.abs(t1 - t0) / scale])
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale)


def test_pn_limiter():
    dim, n, order = 2, (9, 7), 5
    gpu, ref = pair(dim, n, order)
    w0 = pn_state(dim, n, order, seed=12)
    rng = np.random.default_rng(3)
    sel = rng.random(w0.shape[0]) < 0.4
    w0[sel, 0, 1:] += 0.6 * rng.standard_normal((int(sel.sum()), w0.shape[2] - 1))
    wr, nchg = ref.limit(w0)
    assert nchg >= 3
    w = torch.tensor(w0, device="cuda")
    gpu.limit(w)
    wg = w.cpu().numpy()
    np.testing.assert_array_equal(np.any(wg != w0, axis=(1, 2)), np.any(wr != w0, axis=(1, 2)))
    e = state_err(wg, wr, dim, mom_scale=momentum_scale(ref, wr))
    say("  limiter state err %.2e" % e)
    assert e <= 1e-12


def test_pn_driving_projection():
    dim, n, order = 3, (5, 4, 4), 4
    h = 1.0 / n[0]
    drv = dg.Driving(dim, n, order, kmax=3, hi=[n[a] * h for a in range(dim)], basis=1)
    kv = drv.modes()
    drv.update(W.ou_noise(len(kv), 1, seed=5)[0], math.inf)
    s = drv.project().cpu().numpy().reshape(-1, dim, drv.nmodes)
    prob = O.Problem(dim, n, h, order, 1.4, basis=1)
    ref = O.forcing_project(prob, (0.0, 0.0, 0.0), kv, drv.amplitudes())[:, :dim]
    e = np.abs(s - ref).max() / np.abs(ref).max()
    say("  P_n projection err %.2e" % e)
    assert e <= 1e-13


def restrict_pn(q, dim, order):
    """Tensor-basis coefficients [cell][field][p^d] -> the P_n modes in their storage order."""
    degq = O.mode_degrees(order, dim, 0)
    degp = O.mode_degrees(order, dim, 1)
    idx = [int(np.nonzero((degq == d).all(axis=1))[0][0]) for d in degp]
    return np.ascontiguousarray(q[:, :, idx])


@pytest.mark.parametrize("dim,n,order,bc", [(2, (11, 7), 3, None), (2, (9, 8), 6, (2, 0)), (3, (4, 3, 3), 4, None)])
def test_pn_av_rhs_and_steps(dim, n, order, bc):
    """Artificial viscosity on P_n (Sec. 4.1 with the basis of Sec. 2.3; top
    modes = total degree n): the RHS with a nonzero previous sensor rate (the
    wiggle source) within 1e-12 of the oracle's rounding scale; three SSP-RK
    steps, whose stage 1 stores d ln S/dt, within 1e-12 per field group and
    the stored rates within 1e-10 of their maximum."""
    say("P_n AV", dim, n, order, bc)
    h = 1.0 / n[0]
    av = {"f_v": 2.5, "f_w": 0.2}
    ref = O.Problem(dim, n, h, order, 1.4, nu=3e-3, kappa=3e-3, bc=bc, av=av, basis=1)
    gpu = dg.Solver(dim, n, order, 1.4, nu=3e-3, kappa=3e-3, hi=[n[a] * h for a in range(dim)], bc=bc, av=av,
                    basis=1)
    q = W.random_smooth(dim, n, order, nfields=ref.nfields, seed=order + 50, amp=0.08, alpha_level=0.3,
                        vbase=(0.2, -0.1, 0.1)).numpy()
    w0 = restrict_pn(q, dim, order)
    R = np.linspace(-1.0, 2.0, ref.ncells)
    gpu.set_sensor_rate(torch.tensor(R, device="cuda"))
    L = gpu.rhs(torch.tensor(w0, device="cuda")).cpu().numpy()
    e = rhs_err(L, ref.rhs(w0, R_prev=R), ref.rhs_abs(w0, R_prev=R), dim)
    say("  rhs err / rounding scale %.2e" % e)
    assert e <= 1e-12
    gpu.set_sensor_rate(torch.zeros(ref.ncells, dtype=torch.float64, device="cuda"))
    w = torch.tensor(w0, device="cuda")
    wr, Rr = w0, np.zeros(ref.ncells)
    dt = 0.5 * ref.max_dt(w0)[0]
    for _ in range(3):
        gpu.step(w, dt)
        wr, Rr = ref.step(wr, dt, Rr)
    assert gpu.check() == 0
    es = state_err(w.cpu().numpy(), wr, dim, mom_scale=momentum_scale(ref, wr))
    Rg = gpu.get_sensor_rate().cpu().numpy()
    eR = np.abs(Rg - Rr).max() / max(np.abs(Rr).max(), 1e-300)
    say("  state err %.2e, sensor-rate err %.2e (max |R| %.2e)" % (es, eR, np.abs(Rr).max()))
    assert es <= 1e-12
    assert eR <= 1e-10


@pytest.mark.parametrize("dim,n,order", [(2, (11, 7), 4), (3, (4, 3, 3), 3)])
def test_pn_tracer_rhs_and_steps(dim, n, order):
    """The passive tracer on P_n (Sec. 3.4 with the basis of Sec. 2.3): RHS
    within 1e-12 of the oracle's rounding scale, five steps within 1e-12 per
    field group, the tracer total conserved to FP64 rounding."""
    say("P_n tracer", dim, n, order)
    h = 1.0 / n[0]
    ref = O.Problem(dim, n, h, order, 1.4, nu=3e-3, kappa=3e-3, tracer=True, eta=5e-3, basis=1)
    gpu = dg.Solver(dim, n, order, 1.4, nu=3e-3, kappa=3e-3, hi=[n[a] * h for a in range(dim)], tracer=True,
                    eta=5e-3, basis=1)
    hyd = W.random_smooth(dim, n, order, seed=order + 60, amp=0.08, vbase=(0.2, -0.1, 0.1)).numpy()
    rng = np.random.default_rng(order + 61)
    c = 0.05 * rng.standard_normal(hyd[:, :1, :].shape) * 0.5 ** np.arange(order ** dim)
    c[:, 0, 0] = 0.5 + 0.2 * rng.random(hyd.shape[0])
    q = np.concatenate([hyd, c * hyd[:, :1, :1]], axis=1)
    w0 = restrict_pn(q, dim, order)
    L = gpu.rhs(torch.tensor(w0, device="cuda")).cpu().numpy()
    e = rhs_err(L, ref.rhs(w0), ref.rhs_abs(w0), dim)
    say("  rhs err / rounding scale %.2e" % e)
    assert e <= 1e-12
    w = torch.tensor(w0, device="cuda")
    t0 = np.array(gpu.totals(w))
    wr = w0
    dt = 0.5 * ref.max_dt(w0)[0]
    for _ in range(5):
        gpu.step(w, dt)
        wr, _ = ref.step(wr, dt)
    assert gpu.check() == 0
    es = state_err(w.cpu().numpy(), wr, dim, mom_scale=momentum_scale(ref, wr))
    t1 = np.array(gpu.totals(w))
    drift = abs(t1[-1] - t0[-1]) / abs(t0[-1])
    say("  state err %.2e, tracer-total drift %.1e" % (es, drift))
    assert es <= 1e-12
    assert drift <= 1e-13


def test_pn_limiter_with_av():
    """The positivity limiter on P_n with the AV field (it scales the higher
    weights of every field, alpha included): the same cells change and the
    limited states agree with the oracle to 1e-12."""
    dim, n, order = 2, (9, 7), 4
    h = 1.0 / n[0]
    ref = O.Problem(dim, n, h, order, 1.4, av={}, basis=1)
    gpu = dg.Solver(dim, n, order, 1.4, hi=[n[a] * h for a in range(dim)], av={}, basis=1)
    q = W.random_smooth(dim, n, order, nfields=ref.nfields, seed=77, amp=0.08, alpha_level=0.3,
                        vbase=(0.2, -0.1, 0.1)).numpy()
    w0 = restrict_pn(q, dim, order)
    rng = np.random.default_rng(4)
    sel = rng.random(w0.shape[0]) < 0.4
    w0[sel, 0, 1:] += 0.6 * rng.standard_normal((int(sel.sum()), w0.shape[2] - 1))
    wr, nchg = ref.limit(w0)
    assert nchg >= 3
    w = torch.tensor(w0, device="cuda")
    gpu.limit(w)
    wg = w.cpu().numpy()
    np.testing.assert_array_equal(np.any(wg != w0, axis=(1, 2)), np.any(wr != w0, axis=(1, 2)))
    e = state_err(wg, wr, dim, mom_scale=momentum_scale(ref, wr))
    say("  P_n AV limiter state err %.2e (%d cells changed)" % (e, nchg))
    assert e <= 1e-12
