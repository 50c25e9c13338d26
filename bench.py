"""Throughput benchmark of the DG hot path on one MI355X.

A step is one SSP-RK step of the whole path: the CFL reduction (eq. timestep)
on the device, then every RK stage (face kernel: traces, HLLC, recovery and
viscous face flux; volume kernel: contractions, point fluxes, lift,
projection and the FP64 stage combination).  The state is resident in HBM
before the timed region; nothing leaves the device inside it.

Headline workload: the 3D driven-turbulence box, 128^3 cells on the periodic
unit cube, order p = 4 (64 modes x 5 fields per cell, 671M DOFs), Navier-
Stokes with nu = kappa = 2e-5 and the solenoidal driving source, gamma =
1.0001, FP64 (the largest single-GPU configuration).  The driving field is an
Ornstein-Uhlenbeck process on the modes 1 <= |k| <= 3 (seeded draws): every
ceil(0.01 / dt) steps, inside the timed region, its amplitudes are updated on
the host and re-projected on the device (dg_forcing_update / _project).  Metric: DOF-updates per
second per RK stage, (cells x modes x fields x stages) / time; the median of
five repeats of --steps timed steps after --warmup untimed ones.

Extra objects on the JSON line:
  roofline     dominant kernel (by device time): the stage's algorithmic bytes
               (16 B/DOF at stage 1, 24 B/DOF after, the driving coefficients
               once per stage) over its average duration, measured with HIP
               events on the launch stream around every kernel of the sampled
               steps of the timed region (the last step of each repeat and
               every 5th before it);
  stage_roofline  the whole stage (all kernels and launch gaps): the same
               algorithmic bytes and both kernels' flops over the measured
               time per stage, against the HBM and the ALU peaks;
  cpu_baseline the CPU oracle (plain FP64, OpenMP) on a fixed sample of cells
               of the same state (RHS of the sampled cells), on one host core
               and on all of them, scaled to DOF-updates per RK stage;
  fp32_bulk    the same workload with FP32 bulk arithmetic (FP64 state/RK):
               throughput, its RHS error against the oracle on sampled cells
               and its state difference to the FP64 run after the same steps;
  kh_2d        the 2D shear layer, 256 x 512, p = 4 (FP64 and FP32 bulk);
  sod_av_2d    the AV shock tube, 1024 x 128, p = 6 (Euler + artificial
               viscosity, reflecting walls at the x ends), FP64;
  turbulence_3d_pn  the headline box on the total-degree basis P_n (20 modes
               per field at p = 4 instead of 64; Sec. 2.3), same driving;
  ensemble     48 independent 2D boxes (sides 32..512, orders 2..6) stepped by
               one captured hipGraph (grouped launches for the small boxes),
               against the same steps issued box by box;
  kh_order_sweep  the shear layer at every order p = 2..8, FP64 and FP32 bulk
               (5 timed steps each), with the dominant kernel's roofline.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2208_11131_amd as dg  # noqa: E402
from paper_2208_11131_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
EVENT_EVERY = 5                # per-kernel events on every 5th timed step
FP64_PEAK_TF = 78.6            # MI355X FP64 vector (= FP64 matrix)
FP32_PEAK_TF = 157.3           # MI355X FP32 vector


# ---------------------------------------------------------------------------
# algorithmic work per cell (see the design notes: counts of the method's
# sum-factorised work, not of the implementation's extra data movement)
# ---------------------------------------------------------------------------

def point_flops(dim, ns, av):
    """Flops per volume Gauss point: Euler flux (all directions) and, if on,
    the Navier-Stokes and AV additions (divisions and square roots = 1)."""
    c = 30 if dim == 2 else 45
    if ns:
        c += 70 if dim == 2 else 160
    if av:
        c += 40 if dim == 2 else 55
    return c


def face_point_flops(dim, ns, av):
    c = 80 if dim == 2 else 100              # HLLC
    if ns:
        c += 60 if dim == 2 else 110
    if av:
        c += 15 if dim == 2 else 20
    return c


def vol_flops_per_cell(dim, p, F, Fc, grad, ns, av):
    NP = p ** dim
    mac = dim * F * NP * p                     # modal -> points
    if grad:
        mac += dim * F * NP * p                # collocation gradients
    mac += dim * Fc * NP * p                   # D^T of the fluxes
    mac += 2 * dim * Fc * NP                   # face lift (both faces per axis)
    mac += dim * F * NP * p                    # points -> modal
    return 2 * mac + NP * point_flops(dim, ns, av) + 4 * F * NP


def face_flops_per_cell(dim, p, F, Fc, grad, ns, av):
    """Faces per cell = dim (each face counted once)."""
    K = p ** (dim - 1)
    mac = 2 * Fc * K * p                       # two traces
    narr = 2
    if grad:
        mac += 4 * F * K * p                   # recovery value and normal derivative
        narr = 4
    mac += (dim - 1) * narr * F * K * p        # transverse passes
    if grad:
        mac += (dim - 1) * F * K * p           # transverse derivative
    return dim * (2 * mac + K * face_point_flops(dim, ns, av))


def stage_bytes_per_dof(stages):
    """Algorithmic HBM bytes per DOF of each stage of an SSP-RK step (FP64
    state): the first stage reads the state and writes the next register
    (16 B), every later stage also reads the base register (24 B).  The
    5-stage scheme's fourth stage also keeps a partial sum for the last one;
    that register traffic depends on the storage scheme and is not counted."""
    return [16.0] + [24.0] * (stages - 1)


# ---------------------------------------------------------------------------

def make_workload(name, order, device, precision):
    if name == "kh":
        nx, ny = 256, 512
        w = W.kelvin_helmholtz(order, nx, ny, device=device)
        s = dg.Solver(2, (nx, ny), order, 5.0 / 3.0, nu=1e-4, kappa=1e-4, hi=[1.0, 2.0],
                      precision=precision, cfl=0.5)
        desc = {"workload": "kelvin_helmholtz_2d", "cells": [nx, ny], "order": order, "fields": 4,
                "physics": "navier_stokes nu=kappa=1e-4", "gamma": 5.0 / 3.0}
        return s, w, None, desc, dict(dim=2, ns=True, av=False)
    if name in ("turb", "turb_pn"):
        n = 128
        basis = 1 if name == "turb_pn" else 0
        w, _ = W.turbulence(order, n, device=device)
        if basis == 1:
            # the same initial field restricted to total degree <= n, in the P_n storage order
            keep = [lx + order * (ly + order * lz) for lz in range(order) for ly in range(order - lz)
                    for lx in range(order - ly - lz)]
            w = w[:, :, keep].contiguous()
        s = dg.Solver(3, (n, n, n), order, 1.0001, nu=2e-5, kappa=2e-5, precision=precision, cfl=0.5,
                      basis=basis)
        drv = dg.Driving(3, (n, n, n), order, kmax=3, t_corr=1.0, sigma0=0.5, basis=basis)
        f = torch.empty(s.ncells * 3 * s.nmodes, dtype=torch.float64, device=device)
        noise = W.ou_noise(drv.nm, 1024, seed=2208)
        drv.update(noise[0], math.inf)                       # stationary start
        drv.project(f)
        s.set_forcing(f)
        dt0 = s.max_dt(w)[0]
        every = max(1, int(math.ceil(0.01 / dt0)))            # OU update interval 0.01
        state = {"k": 1, "step": 0}

        def refresh():
            # called before every step of the run (warm-up and timed steps
            # alike): the OU update and projection every `every` steps
            step = state["step"]
            state["step"] += 1
            if step % every == 0:
                drv.update(noise[state["k"] % len(noise)], every * dt0)
                state["k"] += 1
                drv.project(f)
                s.set_forcing(f)                           # the library re-evaluates it at the Gauss points
                return True
            return False
        desc = {"workload": "driven_turbulence_3d" + ("_pn" if basis else ""), "cells": [n, n, n], "order": order,
                "fields": 5, "basis": "P_n (total degree)" if basis else "Q_n (tensor)",
                "modes": s.nmodes, "physics": "navier_stokes nu=kappa=2e-5 + OU driving", "gamma": 1.0001,
                "driving": "OU modes 1<=|k|<=3, update + projection every %d steps" % every}
        return s, w, f, desc, dict(dim=3, ns=True, av=False, refresh=refresh, keep=drv)
    if name == "sod":
        nx, ny = 1024, 128
        w = W.sod(order, nx, ny, device=device)
        s = dg.Solver(2, (nx, ny), order, 1.4, hi=[1.0, ny / nx], bc=[2, 0], av={}, precision=precision,
                      cfl=0.3)
        desc = {"workload": "sod_av_2d", "cells": [nx, ny], "order": order, "fields": 5,
                "physics": "euler + artificial viscosity", "gamma": 1.4}
        return s, w, None, desc, dict(dim=2, ns=False, av=True)
    raise ValueError(name)


def group_err(a, b, dim):
    """max over density / momentum vector / energy of ||a - b||_inf / ||b||_inf."""
    e = 0.0
    for g in ([0], list(range(1, 1 + dim)), [dim + 1]):
        den = np.abs(b[:, g]).max()
        e = max(e, float(np.abs(a[:, g] - b[:, g]).max() / den))
    return e


def measure(name, order, precision, steps, warmup, repeats=1, device="cuda"):
    s, w, f, desc, phys = make_workload(name, order, device, precision)
    dim = phys["dim"]
    stages = 1 if order == 1 else 2 if order == 2 else 3 if order == 3 else 5
    sampled = set(range(steps - 1, -1, -EVENT_EVERY))
    # warm-up; its last len(sampled) steps record per-kernel events, so the
    # event pool is filled before the timed region (read and dropped below)
    refresh = phys.get("refresh")
    for i in range(warmup):
        dg.dg_timing_enable(s.ctx, i >= warmup - len(sampled))
        if refresh:
            refresh()
        s.step_cfl(w)
    dg.dg_timing_enable(s.ctx, False)
    torch.cuda.synchronize()
    # timed region: `repeats` runs of `steps` steps, each bracketed by events
    # on the launch stream.  The per-kernel events (every launch of the
    # sampled steps: the last step and every EVENT_EVERY-th before it) cost
    # about 10 % of a step where they are recorded, so they are recorded on a
    # sample of the steps only.
    dg.dg_timing_read(s.ctx)
    stream = torch.cuda.current_stream()
    runs = []
    wall = 0.0
    updates = 0
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for i in range(steps):
            dg.dg_timing_enable(s.ctx, i in sampled)
            if refresh and refresh():
                updates += 1
            s.step_cfl(w)
        dg.dg_timing_enable(s.ctx, False)
        e1.record(stream)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        runs.append(e0.elapsed_time(e1))
    # with periodic driving updates only some repeats hold one: the mean over
    # the repeats (the whole timed region) carries their cost at its rate
    ms = float(np.mean(runs)) if refresh else float(np.median(runs))
    timing = "%s of %d repeats of %d steps" % ("mean" if refresh else "median", repeats, steps)
    kt = dg.dg_timing_read(s.ctx)
    err = s.check()
    if err != 0:
        raise RuntimeError("the run produced a non-physical or non-finite state: %s" % dg.status_str(err))
    dofs = s.ncells * s.nmodes * s.nfields
    value = dofs * stages * steps / (ms * 1e-3)
    # roofline of the dominant kernel
    p = order
    F, Fc = s.nfields, dim + 2
    grad = phys["ns"] or phys["av"]
    vol_fl = vol_flops_per_cell(dim, p, F, Fc, grad, phys["ns"], phys["av"]) * s.ncells
    face_fl = face_flops_per_cell(dim, p, F, Fc, grad, phys["ns"], phys["av"]) * s.ncells
    bpd = stage_bytes_per_dof(stages)
    vol_bytes = dofs * sum(bpd) / len(bpd)                   # per stage (average over the stages)
    if f is not None:
        vol_bytes += 8.0 * s.ncells * dim * s.nmodes          # driving coefficients
    peak_tf = FP64_PEAK_TF if precision == "fp64" else FP32_PEAK_TF
    ridge = peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9)
    kern = {}
    for k, fl, by in (("vol", vol_fl, vol_bytes), ("face", face_fl, 0.0)):
        tms, n = kt[k]
        if n == 0:
            continue
        avg_s = tms * 1e-3 / n
        if by > 0 and fl / by < ridge:
            kern[k] = {"bound": "hbm", "achieved": by / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "avg_us": avg_s * 1e6, "launches": n, "total_ms": tms,
                       "algorithmic_bytes": by, "algorithmic_flops": fl}
        else:
            kern[k] = {"bound": "alu", "achieved": fl / avg_s / 1e12, "peak": peak_tf, "unit": "TFLOP/s",
                       "avg_us": avg_s * 1e6, "launches": n, "total_ms": tms,
                       "algorithmic_bytes": by, "algorithmic_flops": fl}
        kern[k]["frac"] = kern[k]["achieved"] / kern[k]["peak"]
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    # the whole stage (every kernel and launch gap) against the same counts:
    # algorithmic bytes of the stage (charged to the volume kernel above) and
    # the flops of both kernels, over the measured time per stage
    st_s = ms * 1e-3 / (steps * stages)
    stage = {"us": st_s * 1e6, "algorithmic_bytes": vol_bytes, "algorithmic_flops": vol_fl + face_fl,
             "achieved_gbs": vol_bytes / st_s / 1e9, "frac_hbm": vol_bytes / st_s / 1e9 / HBM_PEAK_GBS,
             "achieved_tflops": (vol_fl + face_fl) / st_s / 1e12,
             "frac_alu": (vol_fl + face_fl) / st_s / 1e12 / peak_tf,
             "bytes_per_dof_by_stage": bpd}
    res = {"value": value, "stage": stage, "ms": ms, "runs_ms": runs, "wall_s": wall, "stages": stages,
           "dofs": dofs, "desc": desc, "steps": steps, "warmup": warmup, "repeats": repeats, "timing": timing,
           "driving_updates_timed": updates,
           "kernels": kern, "dominant": dom, "cfl_ms": kt["cfl"][0], "solver": s, "state": w,
           "forcing": f, "phys": phys}
    return res


def measure_graph(r, steps, repeats):
    """The measured workload's step (device CFL + SSP-RK step) captured once
    into a HIP graph and replayed, continuing from the state of `r`.  A step
    right after a driving-field update runs eagerly instead: that call also
    evaluates the new field at the Gauss points, which a replay does not."""
    s, w, phys = r["solver"], r["state"], r["phys"]
    if phys["av"]:
        return None                      # the sensor-rate buffers alternate per step
    refresh = phys.get("refresh")
    dg.dg_timing_enable(s.ctx, False)
    s.step_cfl(w)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.step_cfl(w)
    stream = torch.cuda.current_stream()
    runs, eager = [], 0
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(steps):
            if refresh and refresh():
                s.step_cfl(w)
                eager += 1
            else:
                g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        runs.append(e0.elapsed_time(e1))
    err = s.check()
    if err != 0:
        raise RuntimeError("the graph replays produced a non-physical or non-finite state: %s" % dg.status_str(err))
    ms = float(np.mean(runs)) if refresh else float(np.median(runs))
    del g
    return {"value": r["dofs"] * r["stages"] * steps / (ms * 1e-3), "ms_per_step": ms / steps,
            "eager_ms_per_step": r["ms"] / r["steps"], "speedup_vs_eager": r["ms"] / r["steps"] / (ms / steps),
            "repeats_ms": runs, "eager_steps_after_driving_updates": eager,
            "timing": "%s of %d repeats of %d steps, one captured step per replay" %
                      ("mean" if refresh else "median", repeats, steps)}


def kernel_record(r):
    d = r["kernels"][r["dominant"]]
    return {"kernel": r["dominant"], "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
            "unit": d["unit"], "frac": d["frac"], "avg_us": d["avg_us"],
            "other_kernels": {k: {kk: v[kk] for kk in ("bound", "achieved", "unit", "frac", "avg_us")}
                              for k, v in r["kernels"].items() if k != r["dominant"]}}


def measure_ensemble(steps, warmup):
    sides, orders = W.ensemble_layout(48)
    ws = [W.ensemble_box(b, sides[b], orders[b], device="cuda") for b in range(48)]
    w2 = [w.clone() for w in ws]
    bt = dg.Batch(2, sides, orders, 5.0 / 3.0, cfl=0.5)
    stages = [1 if p == 1 else 2 if p == 2 else 3 if p == 3 else 5 for p in orders]
    work = sum(w.numel() * s for w, s in zip(ws, stages))
    for _ in range(warmup):
        bt.step(ws)
        for i in range(48):
            bt.box_step_cfl(i, w2[i])
    torch.cuda.synchronize()
    res = {}
    for mode in ("graph", "per_box"):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            if mode == "graph":
                bt.step(ws)
            else:
                for i in range(48):
                    bt.box_step_cfl(i, w2[i])
        e1.record()
        torch.cuda.synchronize()
        res[mode] = e0.elapsed_time(e1) / steps
    for i in range(48):
        if bt.box_check(i) != 0:
            raise RuntimeError("ensemble box %d produced a non-physical state" % i)
    same = all(torch.equal(a, b) for a, b in zip(ws, w2))
    dofs = sum(w.numel() for w in ws)
    return {"value": work / (res["graph"] * 1e-3), "unit": "DOF-updates/s", "ms_per_step": res["graph"],
            "per_box_ms_per_step": res["per_box"], "speedup_vs_per_box": res["per_box"] / res["graph"],
            "boxes": 48, "dofs": dofs, "orders": orders, "sides": sides, "bitwise_equal_to_per_box": same}


def traffic_record(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    key = "%s/%s" % (kernel, workload)
    if key not in rec:
        return None
    h = hashlib.sha256()
    for fn in sorted(os.listdir(os.path.join(ROOT, "paper_2208_11131_amd", "csrc"))):
        h.update(open(os.path.join(ROOT, "paper_2208_11131_amd", "csrc", fn), "rb").read())
    if rec[key].get("src_sha256") != h.hexdigest():
        return None
    return rec[key].get("bytes_per_launch")


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, order, one_core_cells=2048, all_core_cells=16384):
    """The CPU oracle on a fixed sample of cells of the workload's initial
    state: the RHS of every sampled cell (the whole state as input), timed on
    one host core and on all of them; DOF-updates per RK stage = sampled DOFs
    / time (the stage combination itself is a few flops per DOF, not timed)."""
    import oracle as O
    if name == "turb":
        wt, ft = W.turbulence(order, 128, device="cuda")
        w = wt.cpu().numpy()
        prob = O.Problem(3, (128, 128, 128), 1.0 / 128, order, 1.0001, nu=2e-5, kappa=2e-5)
        prob.set_forcing(ft.cpu().numpy())
        del wt, ft
    elif name == "kh":
        w = W.kelvin_helmholtz(order, 256, 512, device="cuda").cpu().numpy()
        prob = O.Problem(2, (256, 512), 1.0 / 256, order, 5.0 / 3.0, nu=1e-4, kappa=1e-4)
    else:
        w = W.sod(order, 1024, 128, device="cuda").cpu().numpy()
        prob = O.Problem(2, (1024, 128), 1.0 / 1024, order, 1.4, av={}, bc=(2, 0), cfl=0.3)
    torch.cuda.empty_cache()
    R = np.zeros(prob.ncells) if prob.av is not None else None
    rng = np.random.default_rng(2208)
    dof_cell = prob.nfields * prob.nmodes
    out = {"unit": "DOF-updates/s per RK stage", "kind": "oracle", "cpu_model": _cpu_model(),
           "nproc": os.cpu_count()}
    all_threads = O.num_threads()
    for key, ncell, nthr in (("one_core", one_core_cells, 1), ("all_cores", all_core_cells, all_threads)):
        cells = np.sort(rng.choice(prob.ncells, size=min(ncell, prob.ncells), replace=False))
        O.set_num_threads(nthr)
        t0 = time.perf_counter()
        prob.rhs_cells(w, cells, R_prev=R)
        el = time.perf_counter() - t0
        out[key] = {"value": len(cells) * dof_cell / el, "cores": O.num_threads(), "seconds": el,
                    "cells": int(len(cells))}
    O.set_num_threads(all_threads)
    out["value"] = out["all_cores"]["value"]
    out["cores"] = out["all_cores"]["cores"]
    out["sample"] = ("RHS of %d (one core) and %d (all cores) seeded random cells of the %s state, "
                     "p = %d, as one RK stage each" % (out["one_core"]["cells"], out["all_cores"]["cells"],
                                                         name, order))
    return out


def fp32_oracle_error(r32, ncell=24):
    """RHS of the FP32-bulk path on the whole state against the oracle on
    sampled cells, relative to the oracle's rounding scale and plainly."""
    import oracle as O
    from oracle.compare import rhs_err, rhs_plain
    s, w, f = r32["solver"], r32["state"], r32["forcing"]
    L = s.rhs(w).cpu().numpy()
    wh = w.cpu().numpy()
    d = r32["desc"]
    if d["workload"] == "driven_turbulence_3d":
        prob = O.Problem(3, tuple(d["cells"]), 1.0 / d["cells"][0], d["order"], 1.0001, nu=2e-5, kappa=2e-5)
        prob.set_forcing(f.cpu().numpy())
    elif d["workload"] == "kelvin_helmholtz_2d":
        prob = O.Problem(2, tuple(d["cells"]), 1.0 / d["cells"][0], d["order"], 5.0 / 3.0, nu=1e-4, kappa=1e-4)
    else:
        return None
    cells = np.sort(np.random.default_rng(7).choice(prob.ncells, size=ncell, replace=False))
    Lr = prob.rhs_cells(wh, cells)
    S = prob.rhs_abs(wh, cells=cells)
    return {"rhs_err_vs_rounding_scale": rhs_err(L[cells], Lr, S, prob.dim),
            "rhs_err_plain_per_group": rhs_plain(L[cells], Lr, prob.dim), "sampled_cells": ncell}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--config", default="turb", choices=["kh", "turb", "turb_pn", "sod"])
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline record")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes 3 times (counter calibration)")
    args = ap.parse_args()
    if args.steps < 1 or args.warmup < 0 or args.repeats < 1:
        print("bench.py needs --steps >= 1, --warmup >= 0 and --repeats >= 1", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8}))
        return
    print("bench: %s p=%d %s, %d warmup + %d x %d timed steps" % (args.config, args.order, args.precision,
                                                                  args.warmup, args.repeats, args.steps),
          file=sys.stderr, flush=True)
    res = measure(args.config, args.order, args.precision, args.steps, args.warmup, args.repeats)
    dom = res["kernels"][res["dominant"]]
    kname = {"vol": "vol_kernel", "face": "face_kernel"}[res["dominant"]]
    roof = {"bound": dom["bound"], "achieved": dom["achieved"], "peak": dom["peak"], "unit": dom["unit"],
            "frac": dom["frac"], "traffic": traffic_record(kname, res["desc"]["workload"]),
            "kernel": kname, "avg_us": dom["avg_us"], "launches": dom["launches"],
            "algorithmic_bytes_per_launch": dom["algorithmic_bytes"],
            "other_kernels": {k: {kk: v[kk] for kk in ("bound", "achieved", "unit", "frac", "avg_us")}
                              for k, v in res["kernels"].items() if k != res["dominant"]}}
    line = {
        "metric": "DOF-updates/sec per RK stage (FP64 vs mixed) at order p; roofline fraction",
        "value": res["value"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms"] / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-bulk/f64-state", "data": "synthetic",
        "config": dict(res["desc"], stages_per_step=res["stages"], dofs=res["dofs"],
                       step="device CFL reduction + full SSP-RK step",
                       timing=res["timing"], driving_updates_timed=res["driving_updates_timed"],
                       repeats_ms=res["runs_ms"]),
        "roofline": roof,
        "stage_roofline": res["stage"],
    }
    name, order = args.config, args.order
    w64 = res["state"].cpu().numpy()
    dim = res["phys"]["dim"]
    nsteps64 = args.warmup + args.steps * args.repeats
    if not args.no_extras:
        print("bench: graph replay", file=sys.stderr, flush=True)
        line["graph_replay"] = measure_graph(res, args.steps, args.repeats)
    del res
    torch.cuda.empty_cache()
    if not args.no_extras:
        print("bench: fp32 bulk", file=sys.stderr, flush=True)
        n32 = max(1, (nsteps64 - 2) // args.repeats)
        r32 = measure(name, order, "fp32", n32, nsteps64 - n32 * args.repeats, args.repeats)
        err = group_err(r32["state"].cpu().numpy(), w64, dim)
        rec = {"value": r32["value"], "ms_per_step": r32["ms"] / n32, "speedup_vs_fp64": r32["value"] / line["value"],
               "state_err_vs_fp64_gpu": err, "after_steps": nsteps64,
               "err_measure": "max over rho/momentum/energy of ||a-b||_inf/||b||_inf",
               "roofline": kernel_record(r32), "stage_roofline": r32["stage"]}
        print("bench: fp32 bulk vs oracle (sampled cells)", file=sys.stderr, flush=True)
        rec["vs_oracle"] = fp32_oracle_error(r32)
        line["fp32_bulk"] = rec
        del r32
        torch.cuda.empty_cache()
        if name == "turb":
            print("bench: total-degree basis", file=sys.stderr, flush=True)
            rp = measure("turb_pn", order, "fp64", 10, 3, 3)
            line["turbulence_3d_pn"] = {"value": rp["value"], "ms_per_step": rp["ms"] / 10, "config": rp["desc"],
                                        "dofs": rp["dofs"], "step_time_vs_tensor_basis": rp["ms"] / 10 /
                                        line["ms_per_step"], "roofline": kernel_record(rp),
                                        "stage_roofline": rp["stage"]}
            del rp
            torch.cuda.empty_cache()
        if name != "kh":
            print("bench: 2D shear layer", file=sys.stderr, flush=True)
            rk = measure("kh", 4, "fp64", 20, 60, 3)
            rk32 = measure("kh", 4, "fp32", 20, 60, 3)
            line["kh_2d"] = {"value": rk["value"], "ms_per_step": rk["ms"] / 20, "config": rk["desc"],
                             "roofline": kernel_record(rk), "stage_roofline": rk["stage"],
                             "fp32_bulk": {"value": rk32["value"], "speedup_vs_fp64": rk32["value"] / rk["value"],
                                           "state_err_vs_fp64_gpu": group_err(rk32["state"].cpu().numpy(),
                                                                              rk["state"].cpu().numpy(), 2)}}
            del rk, rk32
            torch.cuda.empty_cache()
        print("bench: shock tube (AV)", file=sys.stderr, flush=True)
        rs = measure("sod", 6, "fp64", 10, 5, 3)
        line["sod_av_2d"] = {"value": rs["value"], "ms_per_step": rs["ms"] / 10, "config": rs["desc"],
                             "roofline": kernel_record(rs), "stage_roofline": rs["stage"]}
        del rs
        torch.cuda.empty_cache()
        print("bench: ensemble", file=sys.stderr, flush=True)
        line["ensemble"] = measure_ensemble(5, 1)
        torch.cuda.empty_cache()
        print("bench: order sweep", file=sys.stderr, flush=True)
        sweep = {}
        for p in range(2, 9):
            rec = {}
            for prec in ("fp64", "fp32"):
                r = measure("kh", p, prec, 5, 2)
                d = r["kernels"][r["dominant"]]
                rec[prec] = {"value": r["value"], "ms_per_step": r["ms"] / 5,
                             "dominant": r["dominant"], "bound": d["bound"], "frac": d["frac"],
                             "stage_frac_hbm": r["stage"]["frac_hbm"]}
                del r
                torch.cuda.empty_cache()
            sweep[str(p)] = rec
        line["kh_order_sweep"] = sweep
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle, sampled cells)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(name, order)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
