"""GPU side of the driving field (Sec. 7.1): the device projection of the
Ornstein-Uhlenbeck modes on the DG basis against the oracle's quadrature
projection, and driven turbulence steps with the field refreshed between
steps (the update of the seeded OU process, then the projection) against the
oracle doing the same."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle.compare import momentum_scale, state_err
from paper_2208_11131_amd import workloads as W

pytestmark = pytest.mark.gpu

dg = pytest.importorskip("paper_2208_11131_amd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_gpu_layout(s_or, dim):
    """Oracle layout [cell][3][M] -> library layout [cell][dim][M]."""
    return np.ascontiguousarray(s_or[:, :dim, :])


@pytest.mark.parametrize("dim,n,order,lo", [(3, (6, 5, 4), 3, (0.0, 0.0, 0.0)), (3, (4, 4, 4), 4, (0.0, 0.0, 0.0)),
                                            (2, (7, 5), 5, (-0.5, 0.25))])
def test_projection_matches_oracle(dim, n, order, lo):
    say("forcing projection", dim, n, order)
    h = 1.0 / n[0]
    hi = [lo[a] + n[a] * h for a in range(dim)]
    drv = dg.Driving(dim, n, order, kmax=3, t_corr=1.0, sigma0=1.0, lo=list(lo), hi=hi)
    kv = drv.modes()
    noise = W.ou_noise(len(kv), 3, seed=7)
    drv.update(noise[0], math.inf)
    drv.update(noise[1], 0.05)
    s = drv.project().cpu().numpy().reshape(-1, dim, order ** dim)
    prob = O.Problem(dim, n, h, order, 1.4)
    ref = to_gpu_layout(O.forcing_project(prob, lo, kv, drv.amplitudes()), dim)
    e = np.abs(s - ref).max() / np.abs(ref).max()
    say("  max err / max |s| %.2e" % e)
    assert e <= 1e-13


def test_driven_turbulence_steps_with_ou_updates():
    """6^3 cells, p = 4, Navier-Stokes, gamma = 1.0001: 9 steps, the driving
    field updated (dt_ou = 3 steps) and re-projected before steps 1, 4, 7."""
    order, n = 4, 6
    say("driven steps with OU updates")
    w0t, _ = W.turbulence(order, n)
    w0 = w0t.numpy()
    gpu = dg.Solver(3, (n, n, n), order, 1.0001, nu=2e-5, kappa=2e-5)
    ref = O.Problem(3, (n, n, n), 1.0 / n, order, 1.0001, nu=2e-5, kappa=2e-5)
    drv = dg.Driving(3, (n, n, n), order, kmax=3, t_corr=1.0, sigma0=0.5)
    kv = drv.modes()
    noise = W.ou_noise(len(kv), 4, seed=2208)
    a_ref = np.zeros((len(kv), 3, 2))
    w = torch.tensor(w0, device="cuda")
    wr = w0
    s_dev = torch.empty(gpu.ncells * 3 * gpu.nmodes, dtype=torch.float64, device="cuda")
    dt = 0.5 * ref.max_dt(w0)[0]
    for step in range(9):
        if step % 3 == 0:
            k = step // 3
            dtu = math.inf if k == 0 else 3 * dt
            drv.update(noise[k], dtu)
            drv.project(s_dev)
            gpu.set_forcing(s_dev)
            a_ref = O.ou_update(3, kv, a_ref, noise[k], dtu, 1.0, 0.5)
            ref.set_forcing(O.forcing_project(ref, (0.0, 0.0, 0.0), kv, a_ref))
        gpu.step(w, dt)
        wr, _ = ref.step(wr, dt)
    assert gpu.check() == 0
    e = state_err(w.cpu().numpy(), wr, 3, mom_scale=momentum_scale(ref, wr))
    say("  state err after 9 driven steps %.2e" % e)
    assert e <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_set_forcing_reevaluates_each_call(precision, tol):
    """dg_set_forcing evaluates the coefficients at the Gauss points for the
    next RHS: a new field (same device array, new values) after a second
    call, no field after NULL, each matching the oracle (FP64 bar, and the
    FP32-bulk bar of the rounding scale)."""
    from oracle.compare import rhs_err
    order, n = 4, (5, 4, 3)
    h = 1.0 / n[0]
    say("set_forcing re-evaluation", precision)
    gpu = dg.Solver(3, n, order, 1.0001, nu=2e-5, kappa=2e-5, hi=[n[a] * h for a in range(3)], precision=precision)
    ref = O.Problem(3, n, h, order, 1.0001, nu=2e-5, kappa=2e-5)
    w0 = W.random_smooth(3, n, order, seed=11, amp=0.08, vbase=(0.2, -0.1, 0.1)).numpy()
    w = torch.tensor(w0, device="cuda")
    rng = np.random.default_rng(12)
    s_dev = torch.empty(gpu.ncells * 3 * gpu.nmodes, dtype=torch.float64, device="cuda")
    for k in range(2):
        s = rng.normal(0.0, 0.3, (gpu.ncells, 3, gpu.nmodes))
        s_dev.copy_(torch.tensor(s.reshape(-1)))
        gpu.set_forcing(s_dev)
        ref.set_forcing(s)
        e = rhs_err(gpu.rhs(w).cpu().numpy(), ref.rhs(w0), ref.rhs_abs(w0), 3)
        say("  field %d: rhs err / rounding scale %.2e" % (k, e))
        assert e <= tol
    gpu.set_forcing(None)
    ref.set_forcing(None)
    e = rhs_err(gpu.rhs(w).cpu().numpy(), ref.rhs(w0), ref.rhs_abs(w0), 3)
    say("  no field: rhs err / rounding scale %.2e" % e)
    assert e <= tol
