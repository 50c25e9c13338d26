"""The allocation-free time-step entry point (dg_max_dt_noalloc) against the
allocating one (dg_max_dt), through the C ABI: the same maxima and step size,
bit for bit, on two calls in a row, the second on a smaller input (fewer
partial maxima in the shared static scratch than the first call left there)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2208_11131_amd import workloads as W

pytestmark = pytest.mark.gpu

dg = pytest.importorskip("paper_2208_11131_amd")


def _case(dim, n, order, nu, av, seed):
    s = dg.Solver(dim, n, order, 1.4, nu=nu, kappa=nu, av=av)
    F = s.nfields
    w0 = W.random_smooth(dim, n, order, nfields=F, seed=seed, amp=0.08,
                         alpha_level=0.3 if av is not None else 0.0).numpy()
    return s, w0


def test_noalloc_max_dt_matches_allocating_entry_point():
    cases = [(2, (40, 33), 4, 1e-3, None, 3),      # 83 CFL blocks
             (2, (6, 5), 3, 0.0, {}, 4),            # 2 CFL blocks: a smaller input second
             (3, (5, 4, 3), 2, 1e-3, None, 5)]
    for dim, n, order, nu, av, seed in cases:
        s, w0 = _case(dim, n, order, nu, av, seed)
        w = torch.tensor(w0, device="cuda")
        print("noalloc", dim, n, order, flush=True)
        dt, cm, vm = dg.dg_max_dt(s.ctx, w)
        out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        dg.dg_max_dt_noalloc(s.ctx, w, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert got[0] == dt and got[1] == cm and got[2] == vm, (got, (dt, cm, vm))
        # and the oracle's step size (Sec. 2.5 eq. timestep)
        h = 1.0 / n[0]
        ref = O.Problem(dim, n, h, order, 1.4, nu=nu, kappa=nu, av=av)
        dtr = ref.max_dt(w0)[0]
        assert abs(got[0] - dtr) <= 1e-14 * dtr
        del s


def test_noalloc_rejects_bad_arguments():
    s, w0 = _case(2, (8, 8), 2, 0.0, None, 1)
    w = torch.tensor(w0, device="cuda")
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    lib = dg.lib()
    assert lib.dg_max_dt_noalloc(None, dg._V(w.data_ptr()), dg._V(out.data_ptr()), None) == dg.DG_EINVAL
    assert lib.dg_max_dt_noalloc(s.ctx, dg._V(w.data_ptr()), None, None) == dg.DG_EINVAL
    assert lib.dg_max_dt_noalloc(s.ctx, dg._V(w.data_ptr() + 8), dg._V(out.data_ptr()), None) == dg.DG_EINVAL
