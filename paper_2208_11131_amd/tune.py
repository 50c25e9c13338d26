"""Autotuner of the launch tiles, per (dimension, order, precision, physics).

For every configuration it measures, on the GPU, the average device time of
the volume kernel over candidate (cells per block, threads per block) pairs
and of the face kernel over candidate (faces per pencil, threads per block)
pairs, using the library's per-launch event timing, and writes the fastest
pair of each into csrc/dg_tiles.inc, the table dg_init uses for its defaults.
Rebuild the library afterwards (paper_2208_11131_amd/build.py).

Tiles change only the work decomposition, never the result: every cell and
face is computed by exactly one block with the same arithmetic.

    python -m paper_2208_11131_amd.tune [--quick] [--out csrc/dg_tiles.inc]
"""
import argparse
import os
import sys
import time

import torch

from . import Solver, dg_timing_enable, dg_timing_read
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))

# (dim, order, precision, physics) configurations of the workloads
#   physics: 0 Euler, 1 Navier-Stokes, 2 artificial viscosity (3 tracer, 4 / 5 total-degree
#   basis: not tuned here; their rows in dg_tiles.inc are kept by hand)
CONFIGS = ([(2, p, pr, 1) for p in range(2, 9) for pr in (0, 1)] +        # shear layer
           [(2, 6, pr, 2) for pr in (0, 1)] +                             # shock tube
           [(3, 4, pr, 1) for pr in (0, 1)] +                             # 3D turbulence
           [(2, p, 0, 0) for p in range(2, 7)])                           # ensemble boxes


def _state(dim, order, phys):
    """A representative state and the solver arguments for one config."""
    if dim == 3:
        n = 64
        w, f = W.turbulence(order, n, device="cuda")
        return w, f, dict(dim=3, n=(n, n, n), gamma=1.0001, nu=2e-5, kappa=2e-5)
    n = (256, 256)
    if phys == 2:
        w = W.sod(order, 256, 256, device="cuda")
        return w, None, dict(dim=2, n=n, gamma=1.4, av=True, bc=[2, 0])
    w = W.random_smooth(2, n, order, seed=order, device="cuda")
    nu = 1e-4 if phys == 1 else 0.0
    return w, None, dict(dim=2, n=n, gamma=1.4, nu=nu, kappa=nu)


def _time(args, order, prec, w0, f, tiles, steps):
    kw = dict(args)
    dim, n, gamma = kw.pop("dim"), kw.pop("n"), kw.pop("gamma")
    hi = [n[a] / n[0] for a in range(dim)]
    s = Solver(dim, n, order, gamma, hi=hi, precision="fp64" if prec == 0 else "fp32", **kw, **tiles)
    if f is not None:
        s.set_forcing(f)
    w = w0.clone()
    s.step_cfl(w)
    torch.cuda.synchronize()
    dg_timing_enable(s.ctx, True)
    dg_timing_read(s.ctx)
    for _ in range(steps):
        s.step_cfl(w)
    t = dg_timing_read(s.ctx)
    used = s.tiles()
    del s
    avg = {k: t[k][0] / max(1, t[k][1]) for k in ("vol", "face")}
    return avg, used


def candidates_vol(NP):
    out = []
    for C in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64):
        for T in (64, 128, 256, 512):
            if C * NP > 2048 or C * NP < 16:
                continue
            if not (0.25 <= C * NP / T <= 8):
                continue
            out.append((C, T))
    return out


def candidates_face(K):
    out = []
    for C in (2, 3, 4, 6, 8, 12, 16, 24, 32, 48):
        for T in (64, 128, 256, 512):
            if C * K > 1024:
                continue
            if not (0.125 <= C * K / T <= 8):
                continue
            out.append((C, T))
    return out


def tune(configs, steps=3, log=sys.stderr):
    rows = []
    for dim, order, prec, phys in configs:
        w0, f, args = _state(dim, order, phys)
        NP, K = order ** dim, order ** (dim - 1)
        base, used = _time(args, order, prec, w0, f, {}, steps)
        # the built-in choice is a candidate too
        best_v = (base["vol"], used[0], used[1])
        best_f = (base["face"], used[2], used[3])
        for C, T in candidates_vol(NP):
            try:
                t, _ = _time(args, order, prec, w0, f, dict(cells_per_block=C, vol_threads=T), steps)
            except Exception:          # tile does not fit (LDS) for this config
                continue
            if best_v is None or t["vol"] < best_v[0]:
                best_v = (t["vol"], C, T)
        for C, T in candidates_face(K):
            try:
                t, _ = _time(args, order, prec, w0, f, dict(faces_per_block=C, face_threads=T), steps)
            except Exception:
                continue
            if best_f is None or t["face"] < best_f[0]:
                best_f = (t["face"], C, T)
        print("dim %d p %d prec %d phys %d: default vol %.1f us face %.1f us (tiles %s) -> "
              "vol %.1f us (C=%d T=%d) face %.1f us (C=%d T=%d)" %
              (dim, order, prec, phys, base["vol"] * 1e3, base["face"] * 1e3, used,
               best_v[0] * 1e3, best_v[1], best_v[2], best_f[0] * 1e3, best_f[1], best_f[2]),
              file=log, flush=True)
        rows.append((dim, order, prec, phys, 0, best_v[1], best_v[2], best_f[1], best_f[2]))
        del w0, f
        torch.cuda.empty_cache()
    return rows


def write_table(rows, path):
    with open(path, "w") as fh:
        fh.write("// Launch tiles measured on the GPU (written by paper_2208_11131_amd/tune.py).\n")
        fh.write("// {dim, order, precision (0 FP64, 1 FP32 bulk), physics (0 Euler, 1 NS, 2 AV),\n")
        fh.write("//  forcing, vol cells, vol threads, face pencil, face threads}\n")
        for r in rows:
            fh.write("    {%d, %d, %d, %d, %d, %d, %d, %d, %d},\n" % r)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "dg_tiles.inc"))
    ap.add_argument("--quick", action="store_true", help="only the 2D p=4 and 3D p=4 Navier-Stokes configs")
    args = ap.parse_args()
    if not torch.cuda.is_available():
        print("the tuner needs a GPU", file=sys.stderr)
        sys.exit(2)
    cfgs = [c for c in CONFIGS if c[:2] in ((2, 4), (3, 4)) and c[3] == 1] if args.quick else CONFIGS
    t0 = time.time()
    rows = tune(cfgs)
    write_table(rows, args.out)
    print("wrote %s (%d entries, %.0f s)" % (args.out, len(rows), time.time() - t0), file=sys.stderr)


if __name__ == "__main__":
    main()
