"""Throughput benchmark of the DG hot path on one MI355X.

A step is one SSP-RK step of the whole path: the CFL reduction (eq. timestep)
on the device, then every RK stage (face kernel: traces, HLLC, recovery and
viscous face flux; volume kernel: contractions, point fluxes, lift,
projection and the FP64 stage combination).  The state is resident in HBM
before the timed region; nothing leaves the device inside it.

Default workload: the 2D Navier-Stokes Kelvin-Helmholtz shear layer,
256 x 512 cells on [0,1]x[0,2], order p = 4 (16 modes x 4 fields per cell),
nu = kappa = 1e-4, FP64.  Metric: DOF-updates per second per RK stage,
(cells x modes x fields x stages) / time.

Extra objects on the JSON line:
  roofline     dominant kernel (by device time): algorithmic bytes or flops per
               launch over its average duration, measured with HIP events on
               the launch stream around every kernel of the sampled steps of
               the timed region (the last step and every 5th before it);
  stage_roofline  the whole stage (all kernels and launch gaps): the stage's
               algorithmic bytes and both kernels' flops over the measured
               time per stage, against the HBM and the ALU peaks;
  cpu_baseline the CPU oracle (plain FP64, OpenMP) timed on four full RK
               steps of the same workload from its initial state;
  fp32_bulk    the same workload with FP32 bulk arithmetic (FP64 state/RK);
  turbulence_3d  the 3D driven-turbulence box, 128^3, p = 4 (FP64), with its
               own roofline record;
  ensemble     48 independent 2D boxes (sides 32..512, orders 2..6) stepped by
               one captured hipGraph (grouped launches for the small boxes),
               against the same steps issued box by box;
  sod_av_2d    the AV shock tube, 1024 x 128, p = 6 (Euler + artificial
               viscosity, outflow in x), FP64;
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


def stage_arrays(stages):
    """FP64 arrays touched by the volume kernel per stage (reads + writes):
    stage 1 reads cur, writes out; later stages also read the base register;
    the 4th stage of the 5-stage scheme reads one more and writes two."""
    if stages == 1:
        return [2]
    if stages == 2:
        return [2, 3]
    if stages == 3:
        return [2, 3, 3]
    return [2, 3, 3, 5, 3]


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
    if name == "turb":
        n = 128
        w, f = W.turbulence(order, n, device=device)
        s = dg.Solver(3, (n, n, n), order, 1.0001, nu=2e-5, kappa=2e-5, precision=precision, cfl=0.5)
        s.set_forcing(f)
        desc = {"workload": "driven_turbulence_3d", "cells": [n, n, n], "order": order, "fields": 5,
                "physics": "navier_stokes nu=kappa=2e-5 + forcing", "gamma": 1.0001}
        return s, w, f, desc, dict(dim=3, ns=True, av=False)
    if name == "sod":
        nx, ny = 1024, 128
        w = W.sod(order, nx, ny, device=device)
        s = dg.Solver(2, (nx, ny), order, 1.4, hi=[1.0, ny / nx], bc=[1, 0], av={}, precision=precision,
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


def run_steps(s, w, n):
    for _ in range(n):
        s.step_cfl(w)


def measure(name, order, precision, steps, warmup, device="cuda"):
    s, w, f, desc, phys = make_workload(name, order, device, precision)
    dim = phys["dim"]
    stages = 1 if order == 1 else 2 if order == 2 else 3 if order == 3 else 5
    sampled = set(range(steps - 1, -1, -EVENT_EVERY))
    # warm-up; its last len(sampled) steps record per-kernel events, so the
    # event pool is filled before the timed region (read and dropped below)
    for i in range(warmup):
        dg.dg_timing_enable(s.ctx, i >= warmup - len(sampled))
        s.step_cfl(w)
    dg.dg_timing_enable(s.ctx, False)
    torch.cuda.synchronize()
    # timed region: K steps, events bracket it on the launch stream.  The
    # per-kernel events (every launch of the sampled steps: the last step and
    # every EVENT_EVERY-th before it) cost about 10 % of a step where they are
    # recorded, so they are recorded on a sample of the steps only.
    dg.dg_timing_read(s.ctx)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        dg.dg_timing_enable(s.ctx, i in sampled)
        s.step_cfl(w)
    dg.dg_timing_enable(s.ctx, False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
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
    arrays = stage_arrays(stages)
    vol_bytes = 8.0 * dofs * sum(arrays) / len(arrays)       # per launch (average over the stages)
    if f is not None:
        vol_bytes += 8.0 * s.ncells * dim * s.nmodes          # forcing coefficients
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
             "frac_alu": (vol_fl + face_fl) / st_s / 1e12 / peak_tf}
    res = {"value": value, "stage": stage, "ms": ms, "wall_s": wall, "stages": stages, "dofs": dofs, "desc": desc, "steps": steps + warmup,
           "kernels": kern, "dominant": dom, "cfl_ms": kt["cfl"][0], "solver": s, "state": w,
           "forcing": f}
    return res


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


def cpu_baseline(desc, order, stages, dofs, nsteps=4):
    """nsteps full RK steps of the CPU oracle from the workload's initial state
    (about 10 s of CPU work on the host's cores)."""
    import oracle as O
    if desc["workload"] != "kelvin_helmholtz_2d":
        return None
    nx, ny = desc["cells"]
    w = W.kelvin_helmholtz(order, nx, ny, device="cpu").numpy()
    prob = O.Problem(2, (nx, ny), 1.0 / nx, order, 5.0 / 3.0, nu=1e-4, kappa=1e-4)
    el = 0.0
    for _ in range(nsteps):
        dt = prob.max_dt(w)[0]
        t0 = time.perf_counter()
        w, _ = prob.step(w, dt)
        el += time.perf_counter() - t0
    return {"value": dofs * stages * nsteps / el, "unit": "DOF-updates/s per RK stage", "cores": O.num_threads(),
            "kind": "oracle", "seconds": el,
            "sample": "%d full SSP-RK steps (%d stages each) of the %dx%d p=%d shear layer from its initial state"
                      % (nsteps, stages, nx, ny, order)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--config", default="kh", choices=["kh", "turb", "sod"])
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the fp32_bulk and turbulence_3d records")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes 3 times (counter calibration)")
    args = ap.parse_args()
    if args.steps < 1 or args.warmup < 0:
        print("bench.py needs --steps >= 1 and --warmup >= 0", file=sys.stderr)
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
    print("bench: %s p=%d %s, %d warmup + %d timed steps" % (args.config, args.order, args.precision, args.warmup,
                                                             args.steps), file=sys.stderr, flush=True)
    res = measure(args.config, args.order, args.precision, args.steps, args.warmup)
    dom = res["kernels"][res["dominant"]]
    kname = {"vol": "vol_kernel", "face": "face_kernel"}[res["dominant"]]
    roof = {"bound": dom["bound"], "achieved": dom["achieved"], "peak": dom["peak"], "unit": dom["unit"],
            "frac": dom["frac"], "traffic": traffic_record(kname, res["desc"]["workload"]),
            "kernel": kname, "avg_us": dom["avg_us"], "launches": dom["launches"],
            "other_kernels": {k: {kk: v[kk] for kk in ("bound", "achieved", "unit", "frac", "avg_us")}
                              for k, v in res["kernels"].items() if k != res["dominant"]}}
    line = {
        "metric": "DOF-updates/sec per RK stage (FP64 vs mixed) at order p; roofline fraction",
        "value": res["value"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms"] / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-bulk/f64-state", "data": "synthetic",
        "config": dict(res["desc"], stages_per_step=res["stages"], dofs=res["dofs"],
                       step="device CFL reduction + full SSP-RK step"),
        "roofline": roof,
        "stage_roofline": res["stage"],
    }
    desc, stages, dofs = res["desc"], res["stages"], res["dofs"]
    w64 = res["state"].cpu().numpy()
    dim = 3 if desc["workload"].endswith("3d") else 2
    del res
    torch.cuda.empty_cache()
    if not args.no_extras:
        print("bench: fp32 bulk", file=sys.stderr, flush=True)
        n32 = args.steps + args.warmup - 2
        r32 = measure(args.config, args.order, "fp32", n32, 2)
        # error of the FP32-bulk state against the FP64 state after the same
        # number of CFL steps from the same initial state
        err = group_err(r32["state"].cpu().numpy(), w64, dim)
        line["fp32_bulk"] = {"value": r32["value"], "ms_per_step": r32["ms"] / n32,
                             "speedup_vs_fp64": r32["value"] / line["value"],
                             "state_err_vs_fp64": err, "after_steps": n32 + 2,
                             "err_measure": "max over rho/momentum/energy of ||a-b||_inf/||b||_inf"}
        del r32
        torch.cuda.empty_cache()
        print("bench: 3D turbulence", file=sys.stderr, flush=True)
        r3 = measure("turb", 4, "fp64", 5, 1)
        d3 = r3["kernels"][r3["dominant"]]
        line["turbulence_3d"] = {"value": r3["value"], "ms_per_step": r3["ms"] / 5, "config": r3["desc"],
                                 "roofline": {"kernel": r3["dominant"], "bound": d3["bound"],
                                              "achieved": d3["achieved"], "peak": d3["peak"], "unit": d3["unit"],
                                              "frac": d3["frac"], "avg_us": d3["avg_us"],
                                              "other_kernels": {k: {kk: v[kk] for kk in
                                                                    ("bound", "achieved", "unit", "frac", "avg_us")}
                                                                for k, v in r3["kernels"].items()
                                                                if k != r3["dominant"]}},
                                 "stage_roofline": r3["stage"]}
        del r3
        torch.cuda.empty_cache()
        print("bench: shock tube (AV)", file=sys.stderr, flush=True)
        rs = measure("sod", 6, "fp64", 5, 1)
        ds = rs["kernels"][rs["dominant"]]
        line["sod_av_2d"] = {"value": rs["value"], "ms_per_step": rs["ms"] / 5, "config": rs["desc"],
                             "roofline": {"kernel": rs["dominant"], "bound": ds["bound"], "achieved": ds["achieved"],
                                          "peak": ds["peak"], "unit": ds["unit"], "frac": ds["frac"],
                                          "avg_us": ds["avg_us"]},
                             "stage_roofline": rs["stage"]}
        del rs
        torch.cuda.empty_cache()
        print("bench: ensemble", file=sys.stderr, flush=True)
        line["ensemble"] = measure_ensemble(5, 1)
        torch.cuda.empty_cache()
        if args.config == "kh":
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
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(desc, args.order, stages, dofs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
