"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Bars (stated per test; error measures in oracle/compare.py, per field group
rho / momentum vector / energy / alpha):
  * FP64 path: dg_rhs within 1e-12 of the oracle's rounding scale S of the
    same sums (per group ||L - Lr||_inf / ||S||_inf; the plain
    ||L - Lr||_inf / ||Lr||_inf is printed next to it); 1 and 10 dg_step's
    within 1e-12 relative to ||w|| (the increments' own relative error is
    printed and bounded by 1e-9); 1e-14 for dg_max_dt and the totals;
  * FP32-bulk path: the bound is stated in the test (measured, see the design
    notes).
Inputs come from the seeded generators of paper_2208_11131_amd.workloads; the
small sizes span several launch tiles and end in a ragged tail.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle.compare import incr_err, momentum_scale, rhs_err, rhs_plain, state_err
from paper_2208_11131_amd import workloads as W

pytestmark = pytest.mark.gpu

dg = pytest.importorskip("paper_2208_11131_amd")

PHYS = {
    "euler": dict(nu=0.0, av=None),
    "ns": dict(nu=3e-3, av=None),
    "av": dict(nu=0.0, av={}),
    "nsav": dict(nu=3e-3, av={"f_v": 2.5, "f_w": 0.2}),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pair(dim, n, order, gamma=1.4, nu=0.0, kappa=None, av=None, bc=None, precision="fp64", cfl=0.5, **kw):
    kappa = nu if kappa is None else kappa
    h = 1.0 / n[0]
    hi = [n[a] * h for a in range(dim)]
    ref = O.Problem(dim, n, h, order, gamma, nu=nu, kappa=kappa, av=av, bc=bc, cfl=cfl)
    gpu = dg.Solver(dim, n, order, gamma, nu=nu, kappa=kappa, hi=hi, bc=bc, av=av, precision=precision,
                    cfl=cfl, **kw)
    return gpu, ref


def relerr(a, b, ref):
    """State error, field groups rho / momentum / energy / alpha."""
    return state_err(a, b, ref.dim, mom_scale=momentum_scale(ref, b))


def rerr(L, Lr, w, ref, R_prev=None, cells=None):
    """RHS error relative to the oracle's rounding scale of the same sums
    (prints the plain per-group relative error too)."""
    S = ref.rhs_abs(w, cells=cells, R_prev=R_prev)
    e = rhs_err(L, Lr, S, ref.dim)
    say("  rhs err / rounding scale %.2e, plain per group %s" % (e, ["%.1e" % x for x in rhs_plain(L, Lr, ref.dim)]))
    return e


def step_ok(wg, wr, w0, ref, tol=1e-12, itol=1e-9):
    """State within tol of ||w|| per group; the increments within itol."""
    e = relerr(wg, wr, ref)
    ie = incr_err(wg, wr, w0, ref.dim)
    say("  state err %.2e, increment err %.2e" % (e, ie))
    return e <= tol and ie <= itol


def state(dim, n, order, prob, seed, vbase=(0, 0, 0)):
    return W.random_smooth(dim, n, order, nfields=prob.nfields, seed=seed, amp=0.08,
                           alpha_level=0.3 if prob.av is not None else 0.0, vbase=vbase).numpy()


RHS_2D = [(o, ph, bc) for o in range(1, 9) for ph in PHYS for bc in ((0, 0),)] + \
         [(o, ph, (1, 0)) for o in (2, 3, 6) for ph in ("euler", "nsav")] + \
         [(o, ph, bc) for o in (2, 5, 6) for ph in ("euler", "nsav") for bc in ((2, 0), (0, 2))]
RHS_3D = [(o, ph, bc) for o in range(1, 7) for ph in ("euler", "ns", "nsav") for bc in ((0, 0, 0),)] + \
         [(o, "nsav", (0, 1, 0)) for o in (2, 4)] + [(o, "nsav", (2, 0, 2)) for o in (3, 4)]


@pytest.mark.parametrize("order,phys,bc", RHS_2D)
def test_rhs_parity_2d(order, phys, bc):
    n = (23, 13) if order <= 4 else (11, 7)
    say("rhs 2d", order, phys, bc, n)
    gpu, ref = pair(2, n, order, bc=bc, **PHYS[phys])
    w0 = state(2, n, order, ref, seed=order)
    R = np.linspace(-1, 2, ref.ncells) if ref.av is not None else None
    if R is not None:
        gpu.set_sensor_rate(torch.tensor(R, device="cuda"))
    L = gpu.rhs(torch.tensor(w0, device="cuda")).cpu().numpy()
    Lr = ref.rhs(w0, R_prev=R)
    assert rerr(L, Lr, w0, ref, R_prev=R) <= 1e-12


@pytest.mark.parametrize("order,phys,bc", RHS_3D)
def test_rhs_parity_3d(order, phys, bc):
    n = (5, 4, 3) if order <= 3 else ((3, 3, 2) if order <= 5 else (2, 2, 2))
    say("rhs 3d", order, phys, bc, n)
    gpu, ref = pair(3, n, order, bc=bc, **PHYS[phys])
    w0 = state(3, n, order, ref, seed=10 + order)
    L = gpu.rhs(torch.tensor(w0, device="cuda")).cpu().numpy()
    Rz = np.zeros(ref.ncells) if ref.av is not None else None
    Lr = ref.rhs(w0, R_prev=Rz)
    assert rerr(L, Lr, w0, ref, R_prev=Rz) <= 1e-12


@pytest.mark.parametrize("order", [7, 8])
def test_rhs_parity_3d_high_order(order):
    n = (2, 2, 1)
    say("rhs 3d high", order)
    gpu, ref = pair(3, n, order, **PHYS["ns"])
    w0 = state(3, n, order, ref, seed=20 + order)
    L = gpu.rhs(torch.tensor(w0, device="cuda")).cpu().numpy()
    assert rerr(L, ref.rhs(w0), w0, ref) <= 1e-12


@pytest.mark.parametrize("dim,order,phys", [(2, 2, "ns"), (2, 4, "nsav"), (2, 8, "euler"), (3, 4, "ns"),
                                            (3, 2, "nsav")])
def test_rhs_fp32_bulk(dim, order, phys):
    n = (17, 9) if dim == 2 else (4, 3, 3)
    say("rhs fp32", dim, order, phys)
    gpu, ref = pair(dim, n, order, precision="fp32", **PHYS[phys])
    w0 = state(dim, n, order, ref, seed=30 + order)
    L = gpu.rhs(torch.tensor(w0, device="cuda")).cpu().numpy()
    Rz = np.zeros(ref.ncells) if ref.av is not None else None
    Lr = ref.rhs(w0, R_prev=Rz)
    assert rerr(L, Lr, w0, ref, R_prev=Rz) <= 1e-5


@pytest.mark.parametrize("dim,order,phys,nsteps", [(2, 1, "euler", 10), (2, 2, "nsav", 10), (2, 3, "ns", 10),
                                                   (2, 4, "nsav", 1), (2, 4, "nsav", 10), (2, 6, "av", 3),
                                                   (3, 2, "ns", 3), (3, 4, "nsav", 2)])
def test_step_parity(dim, order, phys, nsteps):
    n = (12, 9) if dim == 2 else (4, 3, 3)
    say("step", dim, order, phys, nsteps)
    gpu, ref = pair(dim, n, order, bc=(1, 0, 0)[:dim], **PHYS[phys])
    w0 = state(dim, n, order, ref, seed=40 + order)
    dt = 0.5 * ref.max_dt(w0)[0]
    w = torch.tensor(w0, device="cuda")
    wr, Rr = w0, (np.zeros(ref.ncells) if ref.av is not None else None)
    for _ in range(nsteps):
        gpu.step(w, dt)
        wr, Rr = ref.step(wr, dt, Rr)
    assert step_ok(w.cpu().numpy(), wr, w0, ref)
    assert gpu.check() == 0
    if ref.av is not None:
        Rg = gpu.get_sensor_rate().cpu().numpy()
        eR = np.abs(Rg - Rr).max() / max(np.abs(Rr).max(), 1e-300)
        say("  sensor-rate err %.2e (of max |R| = %.2e)" % (eR, np.abs(Rr).max()))
        assert eR <= 1e-10


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 5), (3, 3)])
def test_max_dt_and_totals(dim, order):
    n = (19, 11) if dim == 2 else (5, 4, 3)
    say("dt/totals", dim, order)
    gpu, ref = pair(dim, n, order, cfl=0.3)
    w0 = state(dim, n, order, ref, seed=50 + order)
    w = torch.tensor(w0, device="cuda")
    dt, cm, vm = gpu.max_dt(w)
    dtr, cmr, vmr = ref.max_dt(w0)
    assert abs(dt - dtr) <= 1e-14 * dtr and abs(cm - cmr) <= 1e-14 * cmr and abs(vm - vmr) <= 1e-14 * vmr
    np.testing.assert_allclose(gpu.totals(w), ref.totals(w0), rtol=1e-14, atol=1e-15)


def test_max_dt_many_partial_blocks_and_nan():
    """The CFL reduction over > 4 x 1024 per-block partials: the exact maxima
    (placed in the last cell, i.e. the last partial) and NaN propagation."""
    dim, n, order = 2, (320, 256), 4
    say("dt many blocks")
    gpu, ref = pair(dim, n, order, cfl=0.5, **PHYS["euler"])
    w0 = state(dim, n, order, ref, seed=57)
    w0[-1, dim + 1, 0] *= 3.0                 # hotter last cell: c_max lives in the last partial
    w = torch.tensor(w0, device="cuda")
    dt, cm, vm = gpu.max_dt(w)
    dtr, cmr, vmr = ref.max_dt(w0)
    assert abs(cm - cmr) <= 1e-14 * cmr and abs(vm - vmr) <= 1e-14 * vmr and abs(dt - dtr) <= 1e-14 * dtr
    wn = w0.copy()
    wn[n[0] * n[1] // 2, 0, 3] = float("nan")
    dtn, cmn, _ = gpu.max_dt(torch.tensor(wn, device="cuda"))
    assert np.isnan(dtn) and np.isnan(cmn)


def test_step_cfl_uses_device_dt():
    dim, n, order = 2, (13, 9), 3
    say("step_cfl")
    gpu, ref = pair(dim, n, order, cfl=0.3, **PHYS["ns"])
    w0 = state(dim, n, order, ref, seed=60)
    w = torch.tensor(w0, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    gpu.step_cfl(w, dt_dev)
    dtr = ref.max_dt(w0)[0]
    assert abs(dt_dev.item() - dtr) <= 1e-14 * dtr
    wr, _ = ref.step(w0, dt_dev.item())
    assert step_ok(w.cpu().numpy(), wr, w0, ref)


def test_density_wave_full_run():
    """2D Euler density wave, 16x16, p = 3, SSPRK(3,3), CFL 0.3, to t = 0.1:
    GPU run equals the oracle run, and both approximate the exact wave."""
    order, n, T = 3, 16, 0.1
    say("density wave full run")
    gpu, ref = pair(2, (n, n), order, gamma=5.0 / 3.0, cfl=0.3)
    w0 = W.density_wave(order, n).numpy()
    w = torch.tensor(w0, device="cuda")
    wr = w0
    t = 0.0
    nstep = 0
    while t < T - 1e-14:
        dt = min(ref.max_dt(wr)[0], T - t)
        gdt = gpu.max_dt(w)[0]
        assert abs(gdt - ref.max_dt(wr)[0]) <= 1e-13 * gdt
        gpu.step(w, dt)
        wr, _ = ref.step(wr, dt)
        t += dt
        nstep += 1
    assert 85 <= nstep <= 95
    wg = w.cpu().numpy()
    assert relerr(wg, wr, ref) <= 1e-12
    ex = W.density_wave_exact(order, n, T).numpy()
    assert np.abs(wg[:, 0] - ex[:, 0]).max() < 5e-5


@pytest.mark.parametrize("order", [2, 4, 8])
def test_kelvin_helmholtz_reduced(order):
    """Shear-layer configuration at reduced size (16 x 32), 1 step."""
    nx, ny = 16, 32
    say("KH reduced", order)
    gpu, ref = pair(2, (nx, ny), order, gamma=5.0 / 3.0, nu=1e-4)
    w0 = W.kelvin_helmholtz(order, nx, ny).numpy()
    w = torch.tensor(w0, device="cuda")
    L = gpu.rhs(w).cpu().numpy()
    assert rerr(L, ref.rhs(w0), w0, ref) <= 1e-12
    dt = ref.max_dt(w0)[0]
    gpu.step(w, dt)
    wr, _ = ref.step(w0, dt)
    assert step_ok(w.cpu().numpy(), wr, w0, ref)


def test_sod_reduced_and_y_uniform():
    """Sod configuration (p = 6, AV on, reflecting x ends) on 48 x 1 against
    the oracle for 5 steps; the 48 x 6 strip equals the 48 x 1 strip row by row."""
    order, nx = 6, 48
    say("sod reduced")
    gpu, ref = pair(2, (nx, 1), order, gamma=1.4, av={}, bc=(2, 0), cfl=0.3)
    g6, _ = pair(2, (nx, 6), order, gamma=1.4, av={}, bc=(2, 0), cfl=0.3)
    w0 = W.sod(order, nx, 1).numpy()
    w = torch.tensor(w0, device="cuda")
    w6 = torch.tensor(W.sod(order, nx, 6).numpy(), device="cuda")
    wr, Rr = w0, np.zeros(ref.ncells)
    for _ in range(5):
        dt = ref.max_dt(wr)[0]
        gpu.step(w, dt)
        g6.step(w6, dt)
        wr, Rr = ref.step(wr, dt, Rr)
    assert relerr(w.cpu().numpy(), wr, ref) <= 1e-12
    a6 = w6.cpu().numpy().reshape(6, nx, ref.nfields, -1)
    for j in range(6):
        np.testing.assert_allclose(a6[j], w.cpu().numpy(), rtol=0, atol=1e-13)


def test_turbulence_reduced_with_forcing():
    """3D driven-turbulence configuration at 6^3, p = 4, with the forcing field."""
    order, n = 4, 6
    say("turbulence reduced")
    w0t, s0t = W.turbulence(order, n)
    w0, s0 = w0t.numpy(), s0t.numpy()
    gpu, ref = pair(3, (n, n, n), order, gamma=1.0001, nu=2e-5)
    ref.set_forcing(s0)
    st = torch.tensor(s0, device="cuda")
    gpu.set_forcing(st)
    w = torch.tensor(w0, device="cuda")
    L = gpu.rhs(w).cpu().numpy()
    assert rerr(L, ref.rhs(w0), w0, ref) <= 1e-12
    dt = ref.max_dt(w0)[0]
    gpu.step(w, dt)
    wr, _ = ref.step(w0, dt)
    assert step_ok(w.cpu().numpy(), wr, w0, ref)


def test_ensemble_boxes_reduced():
    """Boxes of the batched ensemble (own size/order each), per-box steps."""
    sides, orders = W.ensemble_layout(48)
    say("ensemble boxes")
    for b in range(3):
        side, order = 16, orders[b]
        gpu, ref = pair(2, (side, side), order, gamma=5.0 / 3.0)
        w0 = W.ensemble_box(b, side, order).numpy()
        w = torch.tensor(w0, device="cuda")
        dt = ref.max_dt(w0)[0]
        gpu.step(w, dt)
        wr, _ = ref.step(w0, dt)
        assert relerr(w.cpu().numpy(), wr, ref) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,order,phys", [(2, 3, "ns"), (3, 2, "nsav"), (2, 4, "nsav"), (3, 4, "ns")])
def test_conservation_gpu(dim, order, phys, precision):
    """Ten periodic steps keep the mass, momentum and energy totals to FP64
    rounding, with an FP64 and with an FP32 bulk (the cell-mean RHS is the
    FP64 sum of the single-valued face fluxes)."""
    n = (16, 12) if dim == 2 else (6, 5, 4)
    say("conservation", dim, order, phys, precision)
    gpu, ref = pair(dim, n, order, precision=precision, **PHYS[phys])
    w0 = state(dim, n, order, ref, seed=70)
    w = torch.tensor(w0, device="cuda")
    t0 = np.array(gpu.totals(w))
    dt = 0.5 * ref.max_dt(w0)[0]
    for _ in range(10):
        gpu.step(w, dt)
    assert gpu.check() == 0
    t1 = np.array(gpu.totals(w))
    scale = np.abs(t0) + np.abs(t0).max()
    say("  drift / scale", ["%.1e" % x for x in np.abs(t1 - t0) / scale])
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale), (t0, t1)


def test_deterministic_and_tile_independent():
    dim, n, order = 2, (21, 11), 4
    say("determinism")
    g1, ref = pair(dim, n, order, **PHYS["nsav"])
    g2, _ = pair(dim, n, order, cells_per_block=3, faces_per_block=5, **PHYS["nsav"])
    w0 = state(dim, n, order, ref, seed=80)
    a = torch.tensor(w0, device="cuda")
    b = torch.tensor(w0, device="cuda")
    c = torch.tensor(w0, device="cuda")
    dt = 0.5 * ref.max_dt(w0)[0]
    for _ in range(3):
        g1.step(a, dt)
        g2.step(b, dt)
    g3, _ = pair(dim, n, order, **PHYS["nsav"])
    for _ in range(3):
        g3.step(c, dt)
    assert torch.equal(a, c)
    assert torch.equal(a, b)


@pytest.mark.parametrize("dim", [2, 3])
def test_fixed_tile_kernels_match_generic(dim):
    """The default tiles of p = 4 Navier-Stokes run the fixed-tile kernels
    (fused lift and RK, split face flux); explicit other tiles run the generic
    ones.  Both must give the same bits, with and without forcing (3D)."""
    order = 4
    n = (20, 12) if dim == 2 else (6, 5, 4)
    say("fixed vs generic", dim)
    g1, ref = pair(dim, n, order, **PHYS["ns"])
    g2, _ = pair(dim, n, order, cells_per_block=3, faces_per_block=5, vol_threads=128, face_threads=128,
                 **PHYS["ns"])
    assert g1.tiles() != g2.tiles()
    w0 = state(dim, n, order, ref, seed=81)
    a = torch.tensor(w0, device="cuda")
    b = torch.tensor(w0, device="cuda")
    if dim == 3:
        ncell = n[0] * n[1] * n[2]
        frc = torch.tensor(np.random.default_rng(82).normal(0.0, 0.3, (ncell, 3, order ** 3)), device="cuda")
        g1.set_forcing(frc)
        g2.set_forcing(frc)
    dt = 0.5 * ref.max_dt(w0)[0]
    for _ in range(2):
        g1.step(a, dt)
        g2.step(b, dt)
    assert torch.equal(a, b)
    assert torch.equal(g1.rhs(a), g2.rhs(a))


@pytest.mark.parametrize("bc", [(1, 1), (2, 2)])
@pytest.mark.parametrize("n", [(1, 1), (1, 5), (3, 1)])
def test_degenerate_meshes(n, bc):
    order = 3
    say("degenerate", n, bc)
    gpu, ref = pair(2, n, order, bc=bc, **PHYS["nsav"])
    w0 = state(2, n, order, ref, seed=90)
    L = gpu.rhs(torch.tensor(w0, device="cuda")).cpu().numpy()
    Rz = np.zeros(ref.ncells)
    assert rerr(L, ref.rhs(w0, R_prev=Rz), w0, ref, R_prev=Rz) <= 1e-12


def test_error_flags():
    dim, n, order = 2, (8, 8), 2
    say("error flags")
    gpu, ref = pair(dim, n, order)
    w0 = state(dim, n, order, ref, seed=91)
    w = torch.tensor(w0, device="cuda")
    gpu.step(w, 1e-4)
    assert gpu.check() == dg.DG_OK
    bad = w0.copy()
    bad[5, 0, 0] = -1.0                       # negative cell-mean density
    wb = torch.tensor(bad, device="cuda")
    gpu.step(wb, 1e-6)
    assert gpu.check() == dg.DG_ENONPHYSICAL
    assert gpu.check() == dg.DG_OK            # cleared
    nan = w0.copy()
    nan[7, 1, 2] = float("nan")
    wn = torch.tensor(nan, device="cuda")
    gpu.step(wn, 1e-6)
    assert gpu.check() == dg.DG_ENONFINITE
    with pytest.raises(ValueError):
        gpu.step(torch.zeros(5, dtype=torch.float64, device="cuda"), 1e-3)
    with pytest.raises(dg.DgError):
        gpu.step(w, -1.0)
    # a state view 8 bytes off a 16-byte boundary is refused before any launch
    buf = torch.zeros(w.numel() + 1, dtype=torch.float64, device="cuda")
    off = buf[1:].view(w.shape)
    assert off.data_ptr() % 16 == 8
    for call in (lambda: gpu.step(off, 1e-6), lambda: gpu.step_cfl(off), lambda: gpu.rhs(off),
                 lambda: gpu.rhs(w, out=off), lambda: gpu.max_dt(off)):
        with pytest.raises(dg.DgError):
            call()
    assert float(buf.abs().sum()) == 0.0


def _sampled_cells(ncells, nsample, rng):
    idx = set(rng.choice(ncells, size=nsample, replace=False).tolist())
    idx.update([0, ncells - 1])
    return np.array(sorted(idx), dtype=np.int64)


@pytest.mark.parametrize("cfg", ["kh_p4", "kh_p8", "sod_p6", "turb_p4"])
def test_full_size_sampled(cfg):
    """Full-size states in the benchmark's launch configuration: the GPU RHS on
    the whole mesh against the oracle at sampled cells (incl. both ends)."""
    rng = np.random.default_rng(2208)
    say("full size", cfg)
    if cfg in ("kh_p4", "kh_p8"):
        order, n = (4 if cfg == "kh_p4" else 8), (256, 512)
        w = W.kelvin_helmholtz(order, *n, device="cuda")
        gpu, ref = pair(2, n, order, gamma=5.0 / 3.0, nu=1e-4)
    elif cfg == "sod_p6":
        order, n = 6, (1024, 128)
        w = W.sod(order, *n, device="cuda")
        gpu, ref = pair(2, n, order, gamma=1.4, av={}, bc=(2, 0), cfl=0.3)
    else:
        order, n = 4, (128, 128, 128)
        wt, st = W.turbulence(order, 128, device="cuda")
        w = wt
        gpu, ref = pair(3, n, order, gamma=1.0001, nu=2e-5)
        gpu.set_forcing(st)
        ref.set_forcing(st.cpu().numpy())
    L = gpu.rhs(w).cpu().numpy()
    wh = w.cpu().numpy()
    cells = _sampled_cells(ref.ncells, 24, rng)
    Rz = np.zeros(ref.ncells) if ref.av is not None else None
    Lr = ref.rhs_cells(wh, cells, R_prev=Rz)
    assert rerr(L[cells], Lr, wh, ref, R_prev=Rz, cells=cells) <= 1e-12


def test_full_size_headline_step():
    """The benchmark's step itself: one dg_step_cfl (device CFL reduction,
    five SSPRK(5,4) stages) of the full 256 x 512, p = 4 shear layer with the
    default (tuned, fixed-tile) kernels, against one oracle step with its own
    CFL step size, on every cell."""
    order, n = 4, (256, 512)
    say("full size headline step")
    w = W.kelvin_helmholtz(order, *n, device="cuda")
    gpu, ref = pair(2, n, order, gamma=5.0 / 3.0, nu=1e-4)
    w0 = w.cpu().numpy()
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    gpu.step_cfl(w, dt_dev)
    assert gpu.check() == 0
    dtr = ref.max_dt(w0)[0]
    assert abs(float(dt_dev) - dtr) <= 1e-14 * dtr
    wr, _ = ref.step(w0, float(dt_dev))
    assert step_ok(w.cpu().numpy(), wr, w0, ref)


def test_full_size_turbulence_steps_conserve():
    """The 3D benchmark step at full size (128^3, p = 4, default tuned tiles),
    a property that holds at any size: periodic faces cancel in the cell
    means, so two dg_step_cfl steps keep the total mass to rounding with the
    forcing on (it acts on momentum and energy only, Sec. 7) and every
    conserved total with it off; the device dt equals the oracle's CFL step
    of the initial state."""
    order, n = 4, (128, 128, 128)
    say("full size turbulence steps")
    w0, s = W.turbulence(order, 128, device="cuda")
    for forced in (True, False):
        gpu, ref = pair(3, n, order, gamma=1.0001, nu=2e-5)
        if forced:
            gpu.set_forcing(s)
        w = w0.clone()
        t0 = np.array(gpu.totals(w))
        dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        gpu.step_cfl(w, dt_dev)
        if forced:
            # CFL maxima over every Gauss point of the initial state, on the CPU
            dtr = ref.max_dt(w0.cpu().numpy())[0]
            assert abs(float(dt_dev) - dtr) <= 1e-14 * dtr
        gpu.step_cfl(w, dt_dev)
        assert gpu.check() == 0
        t1 = np.array(gpu.totals(w))
        scale = np.abs(t0) + np.abs(t0).max()
        keep = [0] if forced else list(range(5))
        assert np.all(np.abs(t1 - t0)[keep] <= 1e-13 * scale[keep]), (forced, t0, t1)
        del gpu, w
        torch.cuda.empty_cache()


def test_fp32_bulk_density_wave_run():
    """Density wave, full run to t = 0.1 with FP32 bulk arithmetic against
    the FP64 oracle run: mean absolute density-coefficient error <= 1e-6."""
    order, n, T = 3, 16, 0.1
    say("fp32 density wave run")
    gpu, ref = pair(2, (n, n), order, gamma=5.0 / 3.0, cfl=0.3, precision="fp32")
    w0 = W.density_wave(order, n).numpy()
    w = torch.tensor(w0, device="cuda")
    wr = w0
    t = 0.0
    while t < T - 1e-14:
        dt = min(ref.max_dt(wr)[0], T - t)
        gpu.step(w, dt)
        wr, _ = ref.step(wr, dt)
        t += dt
    err = np.abs(w.cpu().numpy()[:, 0] - wr[:, 0]).mean()
    say("fp32 density wave mean |drho| =", err)
    assert err <= 1e-6


@pytest.mark.parametrize("order", [2, 4, 8])
def test_fp32_bulk_kelvin_helmholtz_steps(order):
    """Shear layer (16 x 32), 10 steps in FP32 bulk vs the FP64 oracle."""
    nx, ny = 16, 32
    say("fp32 KH steps", order)
    gpu, ref = pair(2, (nx, ny), order, gamma=5.0 / 3.0, nu=1e-4, precision="fp32")
    w0 = W.kelvin_helmholtz(order, nx, ny).numpy()
    w = torch.tensor(w0, device="cuda")
    wr = w0
    dt = ref.max_dt(w0)[0]
    for _ in range(10):
        gpu.step(w, dt)
        wr, _ = ref.step(wr, dt)
    e = relerr(w.cpu().numpy(), wr, ref)
    say("fp32 KH p=%d 10-step state error %.3e" % (order, e))
    assert e <= 1e-5
