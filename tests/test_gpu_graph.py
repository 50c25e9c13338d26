"""GPU: single-box steps captured into a HIP graph (torch.cuda.CUDAGraph on
the library's stream argument) and replayed, against the same steps launched
eagerly on a second context.  Bar: bitwise equal states and step sizes after
every replay (the replays run the same kernels on the same inputs), with
eager work and synchronisations between the replays."""
import sys

import pytest
import torch

from paper_2208_11131_amd import workloads as W

pytestmark = pytest.mark.gpu
dg = pytest.importorskip("paper_2208_11131_amd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(name):
    if name == "turbulence_3d_forced":
        order, n = 3, 6
        w0, s0 = W.turbulence(order, n)
        mk = lambda: dg.Solver(3, (n, n, n), order, 1.0001, nu=2e-5, kappa=2e-5, cfl=0.5)
        return mk, w0, s0, 1
    if name == "sod_av_2d":
        # the sensor-rate buffers alternate per step: two steps per graph
        order, nx, ny = 3, 32, 4
        w0 = W.sod(order, nx, ny)
        mk = lambda: dg.Solver(2, (nx, ny), order, 1.4, hi=[1.0, ny / nx], bc=[2, 0], av={}, cfl=0.3)
        return mk, w0, None, 2
    if name == "kelvin_helmholtz_2d_fp32":
        order, nx, ny = 4, 8, 16
        w0 = W.kelvin_helmholtz(order, nx, ny)
        mk = lambda: dg.Solver(2, (nx, ny), order, 5.0 / 3.0, nu=1e-4, kappa=1e-4, hi=[1.0, 2.0], cfl=0.5,
                               precision="fp32")
        return mk, w0, None, 1
    raise ValueError(name)


@pytest.mark.parametrize("name", ["turbulence_3d_forced", "sod_av_2d", "kelvin_helmholtz_2d_fp32"])
def test_captured_steps_replay_like_eager(name):
    say("graph", name)
    mk, w0, s0, nper = _case(name)
    se, sg = mk(), mk()
    we = w0.to("cuda").contiguous()
    wg = we.clone()
    dte = torch.zeros(1, dtype=torch.float64, device="cuda")
    dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
    if s0 is not None:
        f = s0.to("cuda").contiguous().view(-1)
        se.set_forcing(f)
        sg.set_forcing(f)
    # one eager step each: evaluates the pending driving field, sets up the contexts
    se.step_cfl(we, dte)
    sg.step_cfl(wg, dtg)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(nper):
            sg.step_cfl(wg, dtg)
    for rep in range(4):
        g.replay()
        for _ in range(nper):
            se.step_cfl(we, dte)
        torch.cuda.synchronize()
        assert torch.equal(wg, we), (name, rep)
        assert torch.equal(dtg, dte), (name, rep)
        assert float((we.abs().sum()).item()) > 0.0           # eager work between the replays
    assert se.check() == 0 and sg.check() == 0


def test_captured_fixed_dt_step():
    """dg_step with a host dt: the step size is a kernel argument, captured by value."""
    say("graph fixed dt")
    order, nx = 3, 8
    w0 = W.density_wave(order, nx)
    mk = lambda: dg.Solver(2, (nx, nx), order, 5.0 / 3.0, cfl=0.3)
    se, sg = mk(), mk()
    we = w0.to("cuda").contiguous()
    wg = we.clone()
    se.step(we, 1e-3)
    sg.step(wg, 1e-3)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sg.step(wg, 1e-3)
    for rep in range(3):
        g.replay()
        se.step(we, 1e-3)
        torch.cuda.synchronize()
        assert torch.equal(wg, we), rep
