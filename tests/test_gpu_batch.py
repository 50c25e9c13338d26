"""GPU: batched ensemble (grouped launches replayed from a hipGraph) against
per-box steps and the CPU oracle.  Bars: batched == per-box results bitwise
(same kernels bodies, same per-box arithmetic); per-box dt and states against
the oracle at 1e-14 / 1e-12 (state measure of oracle/compare.py)."""
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


def test_batch_matches_per_box_and_oracle():
    sides = [8, 16, 8, 12, 16, 8, 10]
    orders = [2, 3, 4, 2, 6, 5, 3]
    say("batch", sides, orders)
    bt = dg.Batch(2, sides, orders, 5.0 / 3.0, cfl=0.5)
    w0 = [W.ensemble_box(b, sides[b], orders[b]).numpy() for b in range(len(sides))]
    wg = [torch.tensor(x, device="cuda") for x in w0]       # graph path
    we = [torch.tensor(x, device="cuda") for x in w0]       # eager grouped path
    for _ in range(3):
        bt.step(wg, use_graph=True)
    dts_g = bt.dts()
    for _ in range(3):
        bt.step(we, use_graph=False)
    for i in range(len(sides)):
        assert torch.equal(wg[i], we[i]), i
        assert bt.box_check(i) == 0
    # per-box launches on the same boxes
    wp = [torch.tensor(x, device="cuda") for x in w0]
    for i in range(len(sides)):
        for _ in range(3):
            bt.box_step_cfl(i, wp[i])
        assert torch.equal(wg[i], wp[i]), i
    # oracle: each box with its own CFL step
    for i in range(len(sides)):
        h = 1.0 / sides[i]
        ref = O.Problem(2, (sides[i], sides[i]), h, orders[i], 5.0 / 3.0, cfl=0.5)
        wr = w0[i]
        for _ in range(3):
            dt = ref.max_dt(wr)[0]
            wr, _ = ref.step(wr, dt)
        assert abs(dts_g[i] - dt) <= 1e-14 * dt
        assert state_err(wg[i].cpu().numpy(), wr, 2, mom_scale=momentum_scale(ref, wr)) <= 1e-12, i


def test_batch_with_large_boxes_matches_per_box():
    """Boxes of at least 65536 cells run their own kernels inside the batched
    step, the others the grouped kernels: every box still equals per-box
    stepping bitwise, in the graph and in the eager path; the large box's dt
    equals the oracle's."""
    sides = [256, 12, 320, 8]
    orders = [2, 3, 2, 4]
    say("batch large", sides, orders)
    bt = dg.Batch(2, sides, orders, 5.0 / 3.0, cfl=0.5)
    w0 = [W.ensemble_box(b, sides[b], orders[b]).numpy() for b in range(len(sides))]
    wg = [torch.tensor(x, device="cuda") for x in w0]
    we = [torch.tensor(x, device="cuda") for x in w0]
    wp = [torch.tensor(x, device="cuda") for x in w0]
    for _ in range(2):
        bt.step(wg, use_graph=True)
        bt.step(we, use_graph=False)
    dts = bt.dts()
    for i in range(len(sides)):
        for _ in range(2):
            bt.box_step_cfl(i, wp[i])
        assert torch.equal(wg[i], wp[i]), i
        assert torch.equal(we[i], wp[i]), i
        assert bt.box_check(i) == 0
    ref = O.Problem(2, (sides[0], sides[0]), 1.0 / sides[0], orders[0], 5.0 / 3.0, cfl=0.5)
    w1 = wp[0].cpu().numpy()
    # dt of the last step was taken on the state after one step: recompute it there
    wh = [torch.tensor(w0[0], device="cuda")]
    bt2 = dg.Batch(2, [sides[0]], [orders[0]], 5.0 / 3.0, cfl=0.5)
    bt2.step(wh)
    dtr = ref.max_dt(wh[0].cpu().numpy())[0]
    assert abs(dts[0] - dtr) <= 1e-14 * dtr
    assert np.isfinite(w1).all()


def test_batch_graph_replays_after_pointer_change():
    sides, orders = [8, 8], [3, 4]
    say("batch pointers")
    bt = dg.Batch(2, sides, orders, 5.0 / 3.0)
    w0 = [W.ensemble_box(b, sides[b], orders[b]).numpy() for b in range(2)]
    a = [torch.tensor(x, device="cuda") for x in w0]
    c = [torch.tensor(x, device="cuda") for x in w0]
    bt.step(a)
    bt.step(a)
    bt.step(c)          # new pointers: recapture
    bt.step(c)
    torch.cuda.synchronize()
    for i in range(2):
        assert torch.equal(a[i], c[i])


def test_batch_rejects_av_and_mixed_dims():
    m2 = dg.make_mesh(2, (4, 4))
    m3 = dg.make_mesh(3, (4, 4, 4))
    with pytest.raises(dg.DgError):
        dg.dg_batch_init([m2, m3], [2, 2], 1.4)
    av = dg.dg_av_defaults()
    with pytest.raises(dg.DgError):
        dg.dg_batch_init([m2], [2], 1.4, av=av)


def test_batch_init_failure_releases_everything():
    """dg_batch_init with a valid first box and an invalid later order fails
    with DG_EINVAL and frees the boxes it had already set up (device memory
    returns to its starting level over repeated attempts)."""
    say("batch init failure leak")
    meshes = [dg.make_mesh(2, (256, 256)), dg.make_mesh(2, (32, 32))]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(12):
        with pytest.raises(dg.DgError) as ei:
            dg.dg_batch_init(meshes, [4, 9], 5.0 / 3.0)
        assert ei.value.code == dg.DG_EINVAL
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    # one 256^2 p = 4 box holds about 25 MB of registers: twelve leaks would be ~300 MB
    assert free0 - free1 < 32 * 2 ** 20, (free0, free1)


def test_binding_rejects_wrong_lengths_before_launch():
    """Short or long tensors never reach the library: the binding checks the
    element counts of the batch's state list, the forcing field and the
    sensor-rate arrays and raises ValueError."""
    say("binding length checks")
    bt = dg.Batch(2, [16, 32], [2, 3], 5.0 / 3.0)
    ws = [torch.ones(16 * 16 * 4 * 4, dtype=torch.float64, device="cuda"),
          torch.ones(32 * 32 * 4 * 9, dtype=torch.float64, device="cuda")]
    with pytest.raises(ValueError):
        bt.step(ws[:1])
    with pytest.raises(ValueError):
        bt.step([ws[0], ws[1][:-4]])
    s3 = dg.Solver(3, (3, 3, 2), 2, 1.4, nu=1e-3, kappa=1e-3)
    with pytest.raises(ValueError):
        s3.set_forcing(torch.zeros(18 * 3 * 8 - 1, dtype=torch.float64, device="cuda"))
    s3.set_forcing(torch.zeros(18 * 3 * 8, dtype=torch.float64, device="cuda"))
    s2 = dg.Solver(2, (5, 4), 3, 1.4, av={})
    with pytest.raises(ValueError):
        s2.set_sensor_rate(torch.zeros(19, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        dg.dg_get_sensor_rate(s2.ctx, torch.zeros(21, dtype=torch.float64, device="cuda"))
    assert dg.dg_shape(s2.ctx) == (2, 3, 20, 5)


def test_batch_step_with_given_dt():
    """dg_batch_step_dt: every box advances by the caller's dt_dev[i] (read on
    the device when the step runs).  Equal bitwise to per-box dg_step with the
    same dt, for grouped and large (own-kernel) boxes; a replay of the captured
    graph picks up new values written into dt_dev; a CFL step afterwards
    (dg_batch_step) captures again and still equals per-box stepping."""
    sides = [8, 12, 256, 8]
    orders = [2, 4, 3, 3]
    say("batch with given dt", sides, orders)
    bt = dg.Batch(2, sides, orders, 5.0 / 3.0, cfl=0.5)
    w0 = [W.ensemble_box(b, sides[b], orders[b]).numpy() for b in range(len(sides))]
    wb = [torch.tensor(x, device="cuda") for x in w0]
    wp = [torch.tensor(x, device="cuda") for x in w0]
    dt = torch.tensor([1e-3, 7e-4, 2e-4, 5e-4], dtype=torch.float64, device="cuda")
    for rep in range(3):
        if rep == 2:
            dt.mul_(0.5)                                      # new values, same array: graph replay
        bt.step_dt(wb, dt, use_graph=True)
        for i in range(len(sides)):
            dg.dg_step(dg.dg_batch_box(bt.b, i), wp[i], float(dt[i]))
        torch.cuda.synchronize()
        for i in range(len(sides)):
            assert torch.equal(wb[i], wp[i]), (rep, i)
    assert bt.dts() == dt.cpu().tolist()
    bt.step(wb, use_graph=True)                               # back to CFL steps
    for i in range(len(sides)):
        bt.box_step_cfl(i, wp[i])
        assert torch.equal(wb[i], wp[i]), i
        assert bt.box_check(i) == 0
    with pytest.raises(ValueError):
        bt.step_dt(wb, dt[:3])
