"""GPU runs of the benchmark configurations.

  * Ten SSP-RK steps of every configuration at reduced size against the
    oracle (FP64, 1e-12 of ||w|| per field group; increments printed):
    the shear layer (16 x 32, p = 2, 4, 8, device CFL steps), the shock tube
    on its full 1024-cell axis as a 1-cell strip (AV state and sensor rates
    too), the driven-turbulence box (6^3, p = 4, forcing) and ensemble boxes
    stepped by the grouped, graph-captured batch path.
  * The shock tube at its full size, 1024 x 128, p = 6: ten steps equal the
    1024 x 1 strip row by row (the problem is y-uniform) to 1e-12.
  * The shock tube run to t = 0.2 (Sec. 4.1 artificial viscosity, CFL 0.3,
    reflecting walls at the x ends): L1(rho) against the exact Riemann
    solution (Toro ch. 4, tests/refsol.py), FP64 at 1024 x 128 (measured
    1.78e-4) and in FP32 bulk (within 3 % of the FP64 error; measured 2.3 %),
    and the first-order fall of L1 over 128 -> 1024 cells on 1-cell strips
    (measured 1.03e-3, 5.6e-4, 3.0e-4, 1.78e-4).  The absolute L1 value is
    not printed in the paper (parity unpinned); the bounds below are the
    measured values with a margin.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle.compare import incr_err, momentum_scale, state_err
from paper_2208_11131_amd import workloads as W
from tests import refsol

pytestmark = pytest.mark.gpu

dg = pytest.importorskip("paper_2208_11131_amd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def errs(wg, wr, w0, ref):
    e = state_err(wg, wr, ref.dim, mom_scale=momentum_scale(ref, wr))
    ie = incr_err(wg, wr, w0, ref.dim)
    say("  state err %.2e, increment err %.2e" % (e, ie))
    return e, ie


@pytest.mark.parametrize("order", [2, 4, 8])
def test_ten_steps_shear_layer_reduced(order):
    nx, ny = 16, 32
    say("10 steps KH", order)
    g = 5.0 / 3.0
    ref = O.Problem(2, (nx, ny), 1.0 / nx, order, g, nu=1e-4, kappa=1e-4)
    gpu = dg.Solver(2, (nx, ny), order, g, nu=1e-4, kappa=1e-4, hi=[1.0, 2.0])
    w0 = W.kelvin_helmholtz(order, nx, ny).numpy()
    w = torch.tensor(w0, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    wr = w0
    for _ in range(10):
        gpu.step_cfl(w, dt_dev)
        dtr = ref.max_dt(wr)[0]
        assert abs(float(dt_dev) - dtr) <= 1e-14 * dtr
        wr, _ = ref.step(wr, float(dt_dev))
    assert gpu.check() == 0
    e, ie = errs(w.cpu().numpy(), wr, w0, ref)
    assert e <= 1e-12 and ie <= 1e-9


def test_ten_steps_shock_tube_strip_and_full_width():
    """1024 x 1 strip: 10 steps against the oracle (state, AV field and the
    per-cell d ln S/dt); 1024 x 128 started from the strip's initial state in
    every row: the same 10 steps give the strip in every row.  (Both start
    from the same bits: the sensor threshold of Sec. 4.1 makes the AV field
    depend discontinuously on the state, so initial states that differ by
    rounding need not stay close.)"""
    order, nx = 6, 1024
    say("10 steps Sod 1024x1 and 1024x128")
    g = 1.4
    ref = O.Problem(2, (nx, 1), 1.0 / nx, order, g, av={}, bc=(2, 0), cfl=0.3)
    gs = dg.Solver(2, (nx, 1), order, g, hi=[1.0, 1.0 / nx], bc=[2, 0], av={}, cfl=0.3)
    gf = dg.Solver(2, (nx, 128), order, g, hi=[1.0, 0.125], bc=[2, 0], av={}, cfl=0.3)
    w0 = W.sod(order, nx, 1).numpy()
    ws = torch.tensor(w0, device="cuda")
    wf = torch.tensor(np.tile(w0, (128, 1, 1)), device="cuda")
    wr, Rr = w0, np.zeros(nx)
    for _ in range(10):
        dt = ref.max_dt(wr)[0]
        gdt = gs.max_dt(ws)[0]
        assert abs(gdt - dt) <= 1e-14 * dt
        gs.step(ws, dt)
        gf.step(wf, dt)
        wr, Rr = ref.step(wr, dt, Rr)
    assert gs.check() == 0 and gf.check() == 0
    a = ws.cpu().numpy()
    e, ie = errs(a, wr, w0, ref)
    assert e <= 1e-12 and ie <= 1e-9
    Rg = gs.get_sensor_rate().cpu().numpy()
    eR = np.abs(Rg - Rr).max() / max(np.abs(Rr).max(), 1e-300)
    say("  sensor-rate err %.2e (max |R| %.2e, cells with R != 0: %d)" % (eR, np.abs(Rr).max(), int((Rr != 0).sum())))
    assert eR <= 1e-10
    full = wf.cpu().numpy().reshape(128, nx, ref.nfields, -1)
    scale = np.abs(a).max(axis=(0, 2))                  # per field
    worst = max(float((np.abs(full[j] - a).max(axis=(0, 2)) / scale).max()) for j in range(128))
    say("  1024x128 rows vs strip: %.2e" % worst)
    assert worst <= 1e-12


def test_ten_steps_turbulence_reduced_forced():
    order, n = 4, 6
    say("10 steps turbulence 6^3")
    w0t, s0t = W.turbulence(order, n)
    w0, s0 = w0t.numpy(), s0t.numpy()
    ref = O.Problem(3, (n, n, n), 1.0 / n, order, 1.0001, nu=2e-5, kappa=2e-5)
    ref.set_forcing(s0)
    gpu = dg.Solver(3, (n, n, n), order, 1.0001, nu=2e-5, kappa=2e-5)
    st = torch.tensor(s0, device="cuda")
    gpu.set_forcing(st)
    w = torch.tensor(w0, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    wr = w0
    for _ in range(10):
        gpu.step_cfl(w, dt_dev)
        wr, _ = ref.step(wr, float(dt_dev))
    assert gpu.check() == 0
    e, ie = errs(w.cpu().numpy(), wr, w0, ref)
    assert e <= 1e-12 and ie <= 1e-9


def test_ten_steps_ensemble_batch_path():
    """Six boxes of the ensemble's orders (sides 16 and 24), stepped 10 times
    by one graph-captured batched step (grouped kernels, per-box device
    CFL step) against per-box oracle steps with the same step sizes."""
    _, orders = W.ensemble_layout(48)
    sides = [16, 24, 16, 24, 16, 24]
    ords = orders[:6]
    say("10 steps ensemble batch", ords)
    g = 5.0 / 3.0
    bt = dg.Batch(2, sides, ords, g, cfl=0.5)
    w0 = [W.ensemble_box(b, sides[b], ords[b]).numpy() for b in range(6)]
    ws = [torch.tensor(x, device="cuda") for x in w0]
    refs = [O.Problem(2, (sd, sd), 1.0 / sd, p, g) for sd, p in zip(sides, ords)]
    wr = list(w0)
    for _ in range(10):
        bt.step(ws)
        dts = bt.dts()
        for b in range(6):
            dtr = refs[b].max_dt(wr[b])[0]
            assert abs(dts[b] - dtr) <= 1e-14 * dtr
            wr[b], _ = refs[b].step(wr[b], dts[b])
    for b in range(6):
        assert bt.box_check(b) == 0
        e, ie = errs(ws[b].cpu().numpy(), wr[b], w0[b], refs[b])
        assert e <= 1e-12 and ie <= 1e-9


# ---------------------------------------------------------------------------
# the shock tube to its end time
# ---------------------------------------------------------------------------

T_END = 0.2


def _run_sod(nx, ny, order=6, precision="fp64"):
    g = 1.4
    s = dg.Solver(2, (nx, ny), order, g, hi=[1.0, ny / nx], bc=[2, 0], av={}, cfl=0.3, precision=precision)
    w = W.sod(order, nx, ny, device="cuda")
    t, nstep = 0.0, 0
    while t < T_END - 1e-14:
        dt = s.max_dt(w)[0]
        if not (dt > 0.0 and math.isfinite(dt)):
            raise AssertionError("non-finite step size after %d steps at t = %.4f" % (nstep, t))
        dt = min(dt, T_END - t)
        s.step(w, dt)
        t += dt
        nstep += 1
    st = s.check()
    assert st == 0, (nstep, dg.status_str(st))
    return w.cpu().numpy(), nstep


def _l1_rho(w, nx, ny, order):
    """L1(rho) per unit length along x with n + 3 Gauss points per axis (the
    initial-condition rule), averaged over the rows."""
    g = 1.4
    nq = order + 2
    xq, wq = np.polynomial.legendre.leggauss(nq)
    V = np.polynomial.legendre.legvander(xq, order - 1) * np.sqrt(2 * np.arange(order) + 1)   # (q, l)
    h = 1.0 / nx
    rho = w[:, 0, :].reshape(ny, nx, order, order)        # (j, i, l_y, l_x)
    vals = np.einsum("jiyx,qx,ry->jirq", rho, V, V)       # (j, i, q_y, q_x)
    xc = (np.arange(nx) + 0.5) * h
    X = (xc[:, None] + 0.5 * h * xq[None, :]).reshape(-1)
    ex = refsol.exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, g, (X - 0.5) / T_END)[0].reshape(nx, nq)
    wts = 0.25 * wq[:, None] * wq[None, :]                # (q_y, q_x), sums to 1
    err = (np.abs(vals - ex[None, :, None, :]) * wts[None, None]).sum(axis=(2, 3))   # (j, i)
    return float(err.mean(axis=0).sum() * h)


def test_shock_tube_full_run_fp64():
    order, nx, ny = 6, 1024, 128
    say("Sod full run FP64 1024x128")
    w, nstep = _run_sod(nx, ny, order)
    l1 = _l1_rho(w, nx, ny, order)
    rows = w.reshape(ny, nx, 5, -1)
    spread = float(np.abs(rows - rows[:1]).max() / np.abs(rows[0]).max())
    say("  %d steps, L1(rho) = %.4e, row spread %.1e" % (nstep, l1, spread))
    assert 5000 <= nstep <= 30000
    assert spread <= 1e-10
    assert l1 < 2.5e-4


def test_shock_tube_full_run_fp32_bulk():
    order, nx, ny = 6, 1024, 128
    say("Sod full run FP32 bulk 1024x128")
    w64, _ = _run_sod(nx, 1, order)                       # FP64 reference on the strip (y-uniform)
    l64 = _l1_rho(w64, nx, 1, order)
    w, nstep = _run_sod(nx, ny, order, precision="fp32")
    l1 = _l1_rho(w, nx, ny, order)
    say("  %d steps, L1(rho) FP32 bulk = %.4e, FP64 = %.4e, ratio %.5f" % (nstep, l1, l64, l1 / l64))
    # measured 1.023 (FP32 rounding of the RHS enters the stage-1 sensor rate
    # and through it the wiggle source of the AV field); bound 3 %
    assert abs(l1 / l64 - 1.0) <= 0.03


def test_shock_tube_l1_converges():
    order = 6
    say("Sod L1 convergence on strips")
    l1 = []
    for nx in (128, 256, 512, 1024):
        w, nstep = _run_sod(nx, 1, order)
        l1.append(_l1_rho(w, nx, 1, order))
        say("  nx %d: %d steps, L1 %.4e" % (nx, nstep, l1[-1]))
    rates = [math.log2(l1[i] / l1[i + 1]) for i in range(3)]
    say("  rates", ["%.2f" % r for r in rates])
    assert all(r > 0.6 for r in rates) and sum(rates) / 3 > 0.8
