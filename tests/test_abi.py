"""Host-side checks of the C-ABI library (no GPU needed): it loads and exports
every entry point declared in include/dg.h, and argument validation that
returns before any device work."""
import ctypes
import os
import re

import pytest

import paper_2208_11131_amd as dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "dg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(dg.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(dg.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    # the binding wraps every declared entry point under the same name
    for s in syms:
        assert s in dg.EXPORTS, s


def test_status_strings_and_defaults():
    if not os.path.exists(dg.LIB_PATH):
        pytest.skip("library not built")
    assert dg.status_str(0) == "ok"
    assert "invalid" in dg.status_str(-1)
    av = dg.dg_av_defaults()
    assert (av.enabled, av.scale, av.f_v, av.f_tau, av.f_w, av.s_onset, av.alpha_max) == \
        (1, 1.0, 2.5, 0.5, 0.2, 1e-4, 1.0)
    o = dg.dg_options_defaults()
    assert (o.precision, o.basis, o.cfl) == (0, 0, 0.5)


@pytest.mark.parametrize("case", ["dim", "order", "gamma", "noncubic", "nu", "bc"])
def test_init_rejects_invalid_arguments(case):
    if not os.path.exists(dg.LIB_PATH):
        pytest.skip("library not built")
    m = dg.make_mesh(2, (4, 4))
    order, gamma, nu = 3, 1.4, 0.0
    if case == "dim":
        m.dim = 4
    elif case == "order":
        order = 9
    elif case == "gamma":
        gamma = 1.0
    elif case == "noncubic":
        m.hi[1] = 2.0
    elif case == "nu":
        nu = -1.0
    elif case == "bc":
        m.bc[0] = 7
    ctx = ctypes.c_void_p()
    r = dg.lib().dg_init(ctypes.byref(m), order, gamma, nu, 0.0, None, None, ctypes.byref(ctx))
    assert r == dg.DG_EINVAL and not ctx.value
    assert dg.lib().dg_rhs(None, None, None, None) == dg.DG_EINVAL
    assert dg.lib().dg_step(None, None, 1.0, None) == dg.DG_EINVAL
    assert dg.lib().dg_limit(None, None, None) == dg.DG_EINVAL
    assert dg.lib().dg_max_dt_noalloc(None, None, None, None) == dg.DG_EINVAL


def test_init_rejects_meshes_beyond_the_index_limit():
    """Cell and face indices are 32-bit on the device: meshes whose face
    spaces exceed 2^31 - 1 entries are refused before any device call, so
    this runs without a GPU."""
    if not os.path.exists(dg.LIB_PATH):
        pytest.skip("library not built")
    for dim, n in ((2, (46341, 46341)), (3, (1291, 1291, 1291))):   # (n + 1)^d > 2^31 - 1
        m = dg.make_mesh(dim, n)
        ctx = ctypes.c_void_p()
        r = dg.lib().dg_init(ctypes.byref(m), 1, 1.4, 0.0, 0.0, None, None, ctypes.byref(ctx))
        assert r == dg.DG_EINVAL and not ctx.value
