"""MI355X discontinuous-Galerkin hydrodynamics (arXiv 2208.11131 hot path).

Thin ctypes binding of ``libdgmi.so`` (the HIP kernels and host runtime behind
the C ABI of ``include/dg.h``).  The functions below carry the same names as
the C entry points and only marshal arguments: torch tensors supply device
memory and streams; every step of the computation runs in the library's
kernels.  There is no fallback: if the library is not built, or no GPU is
visible, the calls raise.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgmi.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EDEVICE, DG_ENONPHYSICAL, DG_ENONFINITE, DG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
DG_ESCRATCH = -7
DG_BC_PERIODIC, DG_BC_OUTFLOW, DG_BC_WALL = 0, 1, 2
DG_PREC_FP64, DG_PREC_FP32_BULK = 0, 1


class DgError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, status_str(code), code))


class dg_mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 3)]


class dg_av_params(ctypes.Structure):
    _fields_ = [("enabled", ctypes.c_int), ("scale", ctypes.c_double), ("f_v", ctypes.c_double),
                ("f_tau", ctypes.c_double), ("f_w", ctypes.c_double), ("s_onset", ctypes.c_double),
                ("alpha_max", ctypes.c_double)]


class dg_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("basis", ctypes.c_int), ("cfl", ctypes.c_double),
                ("cells_per_block", ctypes.c_int), ("faces_per_block", ctypes.c_int),
                ("vol_threads", ctypes.c_int), ("face_threads", ctypes.c_int), ("limiter", ctypes.c_int),
                ("tracer", ctypes.c_int), ("tracer_eta", ctypes.c_double)]


_V = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_SIGS = {
    "dg_av_defaults": (None, [ctypes.POINTER(dg_av_params)]),
    "dg_options_defaults": (None, [ctypes.POINTER(dg_options)]),
    "dg_init": (ctypes.c_int, [ctypes.POINTER(dg_mesh), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.POINTER(dg_av_params), ctypes.POINTER(dg_options),
                               ctypes.POINTER(_V)]),
    "dg_free": (None, [_V]),
    "dg_state_len": (ctypes.c_size_t, [_V]),
    "dg_num_fields": (ctypes.c_int, [_V]),
    "dg_num_conserved": (ctypes.c_int, [_V]),
    "dg_num_modes": (ctypes.c_int, [_V]),
    "dg_shape": (ctypes.c_int, [_V, _I, _I, ctypes.POINTER(ctypes.c_longlong), _I]),
    "dg_rhs": (ctypes.c_int, [_V, _V, _V, _V]),
    "dg_step": (ctypes.c_int, [_V, _V, ctypes.c_double, _V]),
    "dg_step_cfl": (ctypes.c_int, [_V, _V, _V, _V]),
    "dg_max_dt": (ctypes.c_int, [_V, _V, _D, _D, _D, _V]),
    "dg_limit": (ctypes.c_int, [_V, _V, _V]),
    "dg_max_dt_noalloc": (ctypes.c_int, [_V, _V, _V, _V]),
    "dg_conserved_totals": (ctypes.c_int, [_V, _V, _D, _V]),
    "dg_set_forcing": (ctypes.c_int, [_V, _V]),
    "dg_set_sensor_rate": (ctypes.c_int, [_V, _V, _V]),
    "dg_get_sensor_rate": (ctypes.c_int, [_V, _V, _V]),
    "dg_check": (ctypes.c_int, [_V, _V]),
    "dg_get_tiles": (ctypes.c_int, [_V, _I, _I, _I, _I]),
    "dg_timing_enable": (ctypes.c_int, [_V, ctypes.c_int]),
    "dg_timing_read": (ctypes.c_int, [_V, _D, ctypes.POINTER(ctypes.c_longlong), _D,
                                      ctypes.POINTER(ctypes.c_longlong), _D, ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_longlong)]),
    "dg_batch_init": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(dg_mesh), ctypes.POINTER(ctypes.c_int),
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(dg_av_params), ctypes.POINTER(dg_options), ctypes.POINTER(_V)]),
    "dg_batch_free": (None, [_V]),
    "dg_batch_step": (ctypes.c_int, [_V, ctypes.POINTER(_V), ctypes.c_int, _V]),
    "dg_batch_step_dt": (ctypes.c_int, [_V, ctypes.POINTER(_V), _V, ctypes.c_int, _V]),
    "dg_batch_dt": (ctypes.c_int, [_V, _D, _V]),
    "dg_batch_box": (ctypes.c_int, [_V, ctypes.c_int, ctypes.POINTER(_V)]),
    "dg_batch_size": (ctypes.c_int, [_V]),
    "dg_forcing_init": (ctypes.c_int, [ctypes.POINTER(dg_mesh), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, ctypes.POINTER(_V)]),
    "dg_forcing_free": (None, [_V]),
    "dg_forcing_num_modes": (ctypes.c_int, [_V]),
    "dg_forcing_modes": (ctypes.c_int, [_V, _I]),
    "dg_forcing_get_amplitudes": (ctypes.c_int, [_V, _D]),
    "dg_forcing_set_amplitudes": (ctypes.c_int, [_V, _D]),
    "dg_forcing_update": (ctypes.c_int, [_V, _D, ctypes.c_double]),
    "dg_forcing_project": (ctypes.c_int, [_V, _V, _V]),
    "dg_status_str": (ctypes.c_char_p, [ctypes.c_int]),
}
EXPORTS = tuple(_SIGS)
_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdgmi.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(code):
    try:
        return lib().dg_status_str(code).decode()
    except Exception:  # pragma: no cover - library missing
        return "status"


def _chk(code, what):
    if code != DG_OK:
        raise DgError(code, what)


def _stream(stream):
    if stream is None:
        return _V(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return _V(stream.cuda_stream)
    return _V(stream)


def _dptr(t, n=None, writable=False):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError("expected a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if n is not None and t.numel() != n:
        raise ValueError("tensor has %d elements, expected %d" % (t.numel(), n))
    return _V(t.data_ptr())


# ---------------------------------------------------------------------------
# same-name wrappers of the C entry points
# ---------------------------------------------------------------------------

def dg_av_defaults():
    av = dg_av_params()
    lib().dg_av_defaults(ctypes.byref(av))
    return av


def dg_options_defaults():
    o = dg_options()
    lib().dg_options_defaults(ctypes.byref(o))
    return o


def make_mesh(dim, n, lo=None, hi=None, bc=None):
    m = dg_mesh()
    m.dim = dim
    for a in range(3):
        m.n[a] = n[a] if a < dim else 1
        m.lo[a] = (lo[a] if lo is not None else 0.0) if a < dim else 0.0
        m.hi[a] = (hi[a] if hi is not None else 1.0) if a < dim else 1.0
        m.bc[a] = (bc[a] if bc is not None else DG_BC_PERIODIC) if a < dim else 0
    return m


def dg_init(mesh, order, gamma, nu=0.0, kappa=0.0, av=None, opt=None):
    ctx = _V()
    _chk(lib().dg_init(ctypes.byref(mesh), order, gamma, nu, kappa,
                       ctypes.byref(av) if av is not None else None,
                       ctypes.byref(opt) if opt is not None else None, ctypes.byref(ctx)), "dg_init")
    return ctx


def dg_free(ctx):
    lib().dg_free(ctx)


def dg_state_len(ctx):
    return lib().dg_state_len(ctx)


def dg_num_fields(ctx):
    return lib().dg_num_fields(ctx)


def dg_num_conserved(ctx):
    return lib().dg_num_conserved(ctx)


def dg_num_modes(ctx):
    return lib().dg_num_modes(ctx)


def dg_shape(ctx):
    """(dim, order, ncells, nfields) of a context."""
    d, o, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    n = ctypes.c_longlong()
    _chk(lib().dg_shape(ctx, ctypes.byref(d), ctypes.byref(o), ctypes.byref(n), ctypes.byref(f)), "dg_shape")
    return d.value, o.value, n.value, f.value


def dg_rhs(ctx, w, wdot, stream=None):
    n = dg_state_len(ctx)
    _chk(lib().dg_rhs(ctx, _dptr(w, n), _dptr(wdot, n), _stream(stream)), "dg_rhs")


def dg_step(ctx, w, dt, stream=None):
    _chk(lib().dg_step(ctx, _dptr(w, dg_state_len(ctx)), float(dt), _stream(stream)), "dg_step")


def dg_step_cfl(ctx, w, dt_dev=None, stream=None):
    p = _dptr(dt_dev, 1) if dt_dev is not None else None
    _chk(lib().dg_step_cfl(ctx, _dptr(w, dg_state_len(ctx)), p, _stream(stream)), "dg_step_cfl")


def dg_limit(ctx, w, stream=None):
    _chk(lib().dg_limit(ctx, _dptr(w, dg_state_len(ctx)), _stream(stream)), "dg_limit")


def dg_max_dt(ctx, w, stream=None):
    dt, cm, vm = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _chk(lib().dg_max_dt(ctx, _dptr(w, dg_state_len(ctx)), ctypes.byref(dt), ctypes.byref(cm),
                         ctypes.byref(vm), _stream(stream)), "dg_max_dt")
    return dt.value, cm.value, vm.value


def dg_max_dt_noalloc(ctx, w, out, stream=None):
    """out: float64 CUDA tensor of 3 elements, receives (dt, c_max, v_max)."""
    _chk(lib().dg_max_dt_noalloc(ctx, _dptr(w, dg_state_len(ctx)), _dptr(out, 3), _stream(stream)),
         "dg_max_dt_noalloc")


def dg_conserved_totals(ctx, w, stream=None):
    out = (ctypes.c_double * dg_num_conserved(ctx))()
    _chk(lib().dg_conserved_totals(ctx, _dptr(w, dg_state_len(ctx)), out, _stream(stream)),
         "dg_conserved_totals")
    return list(out)


def dg_set_forcing(ctx, s):
    if s is None:
        _chk(lib().dg_set_forcing(ctx, None), "dg_set_forcing")
        return
    dim, order, ncells, _ = dg_shape(ctx)
    _chk(lib().dg_set_forcing(ctx, _dptr(s, ncells * dim * dg_num_modes(ctx))), "dg_set_forcing")


def dg_set_sensor_rate(ctx, R, stream=None):
    _chk(lib().dg_set_sensor_rate(ctx, _dptr(R, dg_shape(ctx)[2]), _stream(stream)), "dg_set_sensor_rate")


def dg_get_sensor_rate(ctx, R, stream=None):
    _chk(lib().dg_get_sensor_rate(ctx, _dptr(R, dg_shape(ctx)[2]), _stream(stream)), "dg_get_sensor_rate")


def dg_check(ctx, stream=None):
    return lib().dg_check(ctx, _stream(stream))


def dg_get_tiles(ctx):
    v = [ctypes.c_int() for _ in range(4)]
    _chk(lib().dg_get_tiles(ctx, *[ctypes.byref(x) for x in v]), "dg_get_tiles")
    return tuple(x.value for x in v)


def dg_timing_enable(ctx, on=True):
    _chk(lib().dg_timing_enable(ctx, 1 if on else 0), "dg_timing_enable")


def dg_timing_read(ctx):
    """{'face': (ms, n), 'vol': (ms, n), 'cfl': (ms, n), 'dropped': k}; synchronises."""
    d = [ctypes.c_double() for _ in range(3)]
    n = [ctypes.c_longlong() for _ in range(4)]
    _chk(lib().dg_timing_read(ctx, ctypes.byref(d[0]), ctypes.byref(n[0]), ctypes.byref(d[1]),
                              ctypes.byref(n[1]), ctypes.byref(d[2]), ctypes.byref(n[2]),
                              ctypes.byref(n[3])), "dg_timing_read")
    return {"face": (d[0].value, n[0].value), "vol": (d[1].value, n[1].value),
            "cfl": (d[2].value, n[2].value), "dropped": n[3].value}


def dg_batch_init(meshes, orders, gamma, nu=0.0, kappa=0.0, av=None, opt=None):
    n = len(meshes)
    arr = (dg_mesh * n)(*meshes)
    ords = (ctypes.c_int * n)(*orders)
    b = _V()
    _chk(lib().dg_batch_init(n, arr, ords, gamma, nu, kappa, ctypes.byref(av) if av is not None else None,
                             ctypes.byref(opt) if opt is not None else None, ctypes.byref(b)), "dg_batch_init")
    return b


def dg_batch_free(b):
    lib().dg_batch_free(b)


def dg_batch_size(b):
    return lib().dg_batch_size(b)


def dg_batch_step(b, ws, use_graph=True, stream=None):
    nbox = dg_batch_size(b)
    if len(ws) != nbox:
        raise ValueError("dg_batch_step: %d state tensors for %d boxes" % (len(ws), nbox))
    ptrs = (_V * nbox)(*[_dptr(w, dg_state_len(dg_batch_box(b, i))) for i, w in enumerate(ws)])
    _chk(lib().dg_batch_step(b, ptrs, 1 if use_graph else 0, _stream(stream)), "dg_batch_step")


def dg_batch_step_dt(b, ws, dt, use_graph=True, stream=None):
    """dt: float64 CUDA tensor of nbox step sizes (read when the step runs)."""
    nbox = dg_batch_size(b)
    if len(ws) != nbox:
        raise ValueError("dg_batch_step_dt: %d state tensors for %d boxes" % (len(ws), nbox))
    ptrs = (_V * nbox)(*[_dptr(w, dg_state_len(dg_batch_box(b, i))) for i, w in enumerate(ws)])
    _chk(lib().dg_batch_step_dt(b, ptrs, _dptr(dt, nbox), 1 if use_graph else 0, _stream(stream)),
         "dg_batch_step_dt")


def dg_batch_dt(b, nbox, stream=None):
    out = (ctypes.c_double * nbox)()
    _chk(lib().dg_batch_dt(b, out, _stream(stream)), "dg_batch_dt")
    return list(out)


def dg_batch_box(b, i):
    c = _V()
    _chk(lib().dg_batch_box(b, i, ctypes.byref(c)), "dg_batch_box")
    return c


class Batch:
    """Ensemble of independent 2D/3D boxes advanced by grouped launches
    replayed from a captured hipGraph (one dg_batch)."""

    def __init__(self, dim, sides, orders, gamma, nu=0.0, kappa=0.0, cfl=0.5):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the DG library runs on the GPU only")
        self.dim = dim
        self.meshes = [make_mesh(dim, [sd] * dim, hi=[1.0] * dim) for sd in sides]
        opt = dg_options_defaults()
        opt.cfl = cfl
        self.orders = list(orders)
        self.sides = list(sides)
        self.b = dg_batch_init(self.meshes, self.orders, gamma, nu, kappa, None, opt)
        self.nbox = len(sides)

    def __del__(self):
        b = getattr(self, "b", None)
        # at interpreter shutdown the module's globals may already be None:
        # then the process is ending and the library's memory goes with it
        if b and dg_batch_free is not None and lib is not None:
            dg_batch_free(b)
            self.b = None

    def step(self, ws, use_graph=True, stream=None):
        dg_batch_step(self.b, ws, use_graph, stream)

    def step_dt(self, ws, dt, use_graph=True, stream=None):
        """One step of every box by the caller's step sizes dt (device tensor)."""
        dg_batch_step_dt(self.b, ws, dt, use_graph, stream)

    def dts(self, stream=None):
        return dg_batch_dt(self.b, self.nbox, stream)

    def box_step_cfl(self, i, w, stream=None):
        """Per-box launch of the same step on box i's own buffers."""
        dg_step_cfl(dg_batch_box(self.b, i), w, None, stream)

    def box_check(self, i, stream=None):
        return dg_check(dg_batch_box(self.b, i), stream)


def dg_forcing_init(mesh, order, kmax, t_corr, sigma0, basis=0):
    f = _V()
    _chk(lib().dg_forcing_init(ctypes.byref(mesh), order, basis, kmax, t_corr, sigma0, ctypes.byref(f)),
         "dg_forcing_init")
    return f


def dg_forcing_free(f):
    lib().dg_forcing_free(f)


def dg_forcing_num_modes(f):
    return lib().dg_forcing_num_modes(f)


def dg_forcing_modes(f):
    import numpy as np
    kv = np.zeros((dg_forcing_num_modes(f), 3), dtype=np.int32)
    _chk(lib().dg_forcing_modes(f, kv.ctypes.data_as(_I)), "dg_forcing_modes")
    return kv


def dg_forcing_get_amplitudes(f):
    import numpy as np
    a = np.zeros((dg_forcing_num_modes(f), 3, 2))
    _chk(lib().dg_forcing_get_amplitudes(f, a.ctypes.data_as(_D)), "dg_forcing_get_amplitudes")
    return a


def _host_modes_array(f, a, what):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (dg_forcing_num_modes(f), 3, 2):
        raise ValueError("%s: expected shape %s, got %s" % (what, (dg_forcing_num_modes(f), 3, 2), a.shape))
    return a


def dg_forcing_set_amplitudes(f, a):
    a = _host_modes_array(f, a, "dg_forcing_set_amplitudes")
    _chk(lib().dg_forcing_set_amplitudes(f, a.ctypes.data_as(_D)), "dg_forcing_set_amplitudes")


def dg_forcing_update(f, noise, dt):
    z = _host_modes_array(f, noise, "dg_forcing_update")
    _chk(lib().dg_forcing_update(f, z.ctypes.data_as(_D), float(dt)), "dg_forcing_update")


def dg_forcing_project(f, s, stream=None):
    _chk(lib().dg_forcing_project(f, _dptr(s), _stream(stream)), "dg_forcing_project")


class Driving:
    """Ornstein-Uhlenbeck driving field of one box (one dg_forcing)."""

    def __init__(self, dim, n, order, kmax=3, t_corr=1.0, sigma0=1.0, lo=None, hi=None, basis=0):
        self.dim, self.order = dim, order
        if hi is None:
            hi = [n[a] / n[0] for a in range(dim)]
        self.mesh = make_mesh(dim, n, lo, hi)
        self.f = dg_forcing_init(self.mesh, order, kmax, t_corr, sigma0, basis)
        self.ncells = 1
        for a in range(dim):
            self.ncells *= n[a]
        self.nm = dg_forcing_num_modes(self.f)
        if basis == 0:
            self.nmodes = order ** dim
        else:
            self.nmodes = order * (order + 1) // 2 if dim == 2 else order * (order + 1) * (order + 2) // 6

    def __del__(self):
        f = getattr(self, "f", None)
        if f and dg_forcing_free is not None and lib is not None:   # see Batch.__del__
            dg_forcing_free(f)
            self.f = None

    def modes(self):
        return dg_forcing_modes(self.f)

    def amplitudes(self):
        return dg_forcing_get_amplitudes(self.f)

    def set_amplitudes(self, a):
        dg_forcing_set_amplitudes(self.f, a)

    def update(self, noise, dt):
        dg_forcing_update(self.f, noise, dt)

    def project(self, out=None, stream=None):
        n = self.ncells * self.dim * self.nmodes
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device="cuda")
        elif out.numel() != n:
            raise ValueError("dg_forcing_project: output has %d elements, expected %d" % (out.numel(), n))
        dg_forcing_project(self.f, out, stream)
        return out


# ---------------------------------------------------------------------------
# convenience object (owns one context)
# ---------------------------------------------------------------------------

class Solver:
    """One DG context on the current GPU.

    ``av``: None (off), True (paper defaults) or a dict overriding defaults.
    ``tracer``/``eta``: the passive tracer field c rho and its diffusivity.
    ``precision``: "fp64" or "fp32" (FP32 bulk, FP64 state and RK)."""

    def __init__(self, dim, n, order, gamma, nu=0.0, kappa=0.0, lo=None, hi=None, bc=None, av=None,
                 precision="fp64", cfl=0.5, cells_per_block=0, faces_per_block=0, vol_threads=0,
                 face_threads=0, limiter=False, tracer=False, eta=0.0, basis=0):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the DG library runs on the GPU only")
        self.dim, self.order = dim, order
        if hi is None:
            hi = [n[a] / n[0] for a in range(dim)]
        self.mesh = make_mesh(dim, n, lo, hi, bc)
        avp = None
        if av is not None and av is not False:
            avp = dg_av_defaults()
            if isinstance(av, dict):
                for k, v in av.items():
                    setattr(avp, k, v)
        opt = dg_options_defaults()
        opt.precision = DG_PREC_FP64 if precision == "fp64" else DG_PREC_FP32_BULK
        opt.cfl = cfl
        opt.cells_per_block = cells_per_block
        opt.faces_per_block = faces_per_block
        opt.vol_threads = vol_threads
        opt.face_threads = face_threads
        opt.limiter = 1 if limiter else 0
        opt.tracer = 1 if tracer else 0
        opt.tracer_eta = eta
        opt.basis = basis
        self.ctx = dg_init(self.mesh, order, gamma, nu, kappa, avp, opt)
        self.nfields = dg_num_fields(self.ctx)
        self.ncells = 1
        for a in range(dim):
            self.ncells *= n[a]
        self.nmodes = dg_num_modes(self.ctx)
        self._forcing = None

    @property
    def shape(self):
        return (self.ncells, self.nfields, self.nmodes)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and dg_free is not None and lib is not None:   # see Batch.__del__
            dg_free(ctx)
            self.ctx = None

    def rhs(self, w, out=None, stream=None):
        out = torch.empty_like(w) if out is None else out
        dg_rhs(self.ctx, w, out, stream)
        return out

    def step(self, w, dt, stream=None):
        dg_step(self.ctx, w, dt, stream)

    def step_cfl(self, w, dt_dev=None, stream=None):
        dg_step_cfl(self.ctx, w, dt_dev, stream)

    def max_dt(self, w, stream=None):
        return dg_max_dt(self.ctx, w, stream)

    def limit(self, w, stream=None):
        dg_limit(self.ctx, w, stream)

    def totals(self, w, stream=None):
        return dg_conserved_totals(self.ctx, w, stream)

    def set_forcing(self, s):
        self._forcing = s
        dg_set_forcing(self.ctx, s)

    def set_sensor_rate(self, R, stream=None):
        dg_set_sensor_rate(self.ctx, R, stream)

    def get_sensor_rate(self, stream=None):
        R = torch.empty(self.ncells, dtype=torch.float64, device="cuda")
        dg_get_sensor_rate(self.ctx, R, stream)
        return R

    def check(self, stream=None):
        return dg_check(self.ctx, stream)

    def tiles(self):
        return dg_get_tiles(self.ctx)
