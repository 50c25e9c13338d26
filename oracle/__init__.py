"""Plain FP64 CPU oracle for the DG right-hand side and SSP-RK step.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product library never imports or calls it.

This module is argument marshalling (ctypes over numpy arrays) around
``libdgoracle.so``, built from ``dg_oracle.c`` by ``build()``.  Every numerical
step lives in the C source, which cites the paper section for each quantity.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libdgoracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
             _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("bc", ctypes.c_int * 3),
        ("h", ctypes.c_double), ("order", ctypes.c_int),
        ("gamma", ctypes.c_double), ("nu", ctypes.c_double), ("kappa", ctypes.c_double),
        ("av_on", ctypes.c_int), ("av_scale", ctypes.c_double), ("f_v", ctypes.c_double),
        ("f_tau", ctypes.c_double), ("f_w", ctypes.c_double), ("s_onset", ctypes.c_double),
        ("alpha_max", ctypes.c_double), ("cfl", ctypes.c_double),
        ("forcing", ctypes.POINTER(ctypes.c_double)),
        ("limiter", ctypes.c_int),
        ("tracer", ctypes.c_int), ("eta", ctypes.c_double),
        ("basis", ctypes.c_int),
    ]


_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(Params)
        sig = {
            "or_legendre": (None, [ctypes.c_int, ctypes.c_double, _D, _D]),
            "or_gauss": (None, [ctypes.c_int, _D, _D]),
            "or_euler_flux": (None, [ctypes.c_int, ctypes.c_double, _D, ctypes.c_int, _D]),
            "or_hllc": (None, [ctypes.c_int, ctypes.c_double, _D, _D, ctypes.c_int, _D]),
            "or_recovery_fraction": (ctypes.c_double, [ctypes.c_int]),
            "or_recover_face": (None, [P, _D, _D, ctypes.c_int, _D, _D]),
            "or_sensor": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, _D]),
            "or_sensor_rate": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, _D, _D]),
            "or_rhs": (None, [P, _D, _D, _D, _D]),
            "or_rhs_cells": (None, [P, _D, _D, ctypes.c_long, ctypes.POINTER(ctypes.c_long), _D]),
            "or_rhs_abs": (None, [P, _D, _D, ctypes.c_long, ctypes.POINTER(ctypes.c_long), _D]),
            "or_max_dt": (ctypes.c_double, [P, _D, _D, _D]),
            "or_rk_stages": (ctypes.c_int, [ctypes.c_int]),
            "or_step": (None, [P, _D, ctypes.c_double, _D]),
            "or_totals": (None, [P, _D, _D]),
            "or_limit": (ctypes.c_long, [P, _D]),
            "or_n_modes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "or_mode_degrees": (None, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int)]),
            "or_forcing_modes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
            "or_ou_update": (None, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D, _D,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double]),
            "or_forcing_project": (None, [P, _D, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D, _D]),
            "or_num_threads": (ctypes.c_int, []),
            "or_set_num_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


class Problem:
    """Mesh, order and physics of one oracle run (mirrors the library's init)."""

    def __init__(self, dim, n, h, order, gamma, nu=0.0, kappa=0.0, bc=None, av=None,
                 cfl=0.5, forcing=None, limiter=False, tracer=False, eta=0.0, basis=0):
        self.dim, self.order = dim, order
        self.n = tuple(n) + (1,) * (3 - len(n))
        self.h = h
        self.p = Params()
        self.p.dim = dim
        for a in range(3):
            self.p.n[a] = self.n[a]
            self.p.bc[a] = (bc[a] if bc is not None and a < len(bc) else 0)
        self.p.h, self.p.order = h, order
        self.p.gamma, self.p.nu, self.p.kappa = gamma, nu, kappa
        self.p.cfl = cfl
        self.p.limiter = 1 if limiter else 0
        self.p.tracer = 1 if tracer else 0
        self.p.eta = eta
        self.p.basis = basis
        self.av = av
        if av is not None:
            self.p.av_on = 1
            self.p.av_scale = av.get("scale", 1.0)
            self.p.f_v = av.get("f_v", 2.5)
            self.p.f_tau = av.get("f_tau", 0.5)
            self.p.f_w = av.get("f_w", 0.2)
            self.p.s_onset = av.get("s_onset", 1e-4)
            self.p.alpha_max = av.get("alpha_max", 1.0)
        self.set_forcing(forcing)
        self.ncons = dim + 2 + (1 if tracer else 0)
        self.nfields = self.ncons + (1 if av is not None else 0)
        self.basis = basis
        if basis == 0:
            self.nmodes = order ** dim
        else:
            self.nmodes = order * (order + 1) // 2 if dim == 2 else order * (order + 1) * (order + 2) // 6
        self.ncells = int(np.prod(self.n[:dim]))

    def set_forcing(self, s):
        self._forcing = None if s is None else np.ascontiguousarray(s, dtype=np.float64)
        self.p.forcing = _ptr(self._forcing)

    @property
    def shape(self):
        return (self.ncells, self.nfields, self.nmodes)

    def rhs(self, w, R_prev=None, want_R=False):
        lib = _load()
        w = np.ascontiguousarray(w, dtype=np.float64)
        out = np.zeros_like(w)
        R_out = np.zeros(self.ncells) if want_R else None
        Rp = None if R_prev is None else np.ascontiguousarray(R_prev, dtype=np.float64)
        lib.or_rhs(ctypes.byref(self.p), _ptr(w), _ptr(Rp), _ptr(out), _ptr(R_out))
        return (out, R_out) if want_R else out

    def rhs_cells(self, w, cells, R_prev=None):
        """RHS of the listed cells only (whole state w as input)."""
        lib = _load()
        w = np.ascontiguousarray(w, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros((len(cells), self.nfields, self.nmodes))
        Rp = None if R_prev is None else np.ascontiguousarray(R_prev, dtype=np.float64)
        lib.or_rhs_cells(ctypes.byref(self.p), _ptr(w), _ptr(Rp), len(cells),
                         cells.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _ptr(out))
        return out

    def rhs_abs(self, w, cells=None, R_prev=None):
        """Rounding scale of the RHS: per coefficient, the sum of the
        magnitudes of the summands of its volume, source and surface sums
        (of the listed cells, or of every cell)."""
        lib = _load()
        w = np.ascontiguousarray(w, dtype=np.float64)
        Rp = None if R_prev is None else np.ascontiguousarray(R_prev, dtype=np.float64)
        if cells is None:
            out = np.zeros_like(w)
            lib.or_rhs_abs(ctypes.byref(self.p), _ptr(w), _ptr(Rp), 0, None, _ptr(out))
        else:
            cells = np.ascontiguousarray(cells, dtype=np.int64)
            out = np.zeros((len(cells), self.nfields, self.nmodes))
            lib.or_rhs_abs(ctypes.byref(self.p), _ptr(w), _ptr(Rp), len(cells),
                           cells.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _ptr(out))
        return out

    def step(self, w, dt, R_state=None):
        """One SSP-RK step; returns (w_new, R_new)."""
        lib = _load()
        w = np.array(w, dtype=np.float64, order="C", copy=True)
        R = None
        if self.av is not None:
            R = (np.zeros(self.ncells) if R_state is None
                 else np.array(R_state, dtype=np.float64, copy=True))
        lib.or_step(ctypes.byref(self.p), _ptr(w), float(dt), _ptr(R))
        return w, R

    def max_dt(self, w):
        lib = _load()
        w = np.ascontiguousarray(w, dtype=np.float64)
        cm, vm = ctypes.c_double(), ctypes.c_double()
        dt = lib.or_max_dt(ctypes.byref(self.p), _ptr(w), ctypes.byref(cm), ctypes.byref(vm))
        return dt, cm.value, vm.value

    def limit(self, w):
        """Positivity limiter (Sec. 4.2) on every cell; returns (w_new, cells changed)."""
        lib = _load()
        w = np.array(w, dtype=np.float64, order="C", copy=True)
        n = lib.or_limit(ctypes.byref(self.p), _ptr(w))
        return w, int(n)

    def totals(self, w):
        lib = _load()
        w = np.ascontiguousarray(w, dtype=np.float64)
        out = np.zeros(self.ncons)
        lib.or_totals(ctypes.byref(self.p), _ptr(w), _ptr(out))
        return out

    def recover_face(self, wL, wR, axis):
        lib = _load()
        K = self.order ** (self.dim - 1)
        ut = np.zeros((K, self.nfields))
        gt = np.zeros((K, self.dim, self.nfields))
        wL = np.ascontiguousarray(wL, dtype=np.float64)
        wR = np.ascontiguousarray(wR, dtype=np.float64)
        lib.or_recover_face(ctypes.byref(self.p), _ptr(wL), _ptr(wR), axis, _ptr(ut), _ptr(gt))
        return ut, gt


def n_modes(order, dim, basis):
    return _load().or_n_modes(order, dim, basis)


def mode_degrees(order, dim, basis):
    """(M, 3) int array of the degrees of every mode of the basis."""
    lib = _load()
    M = lib.or_n_modes(order, dim, basis)
    out = np.zeros((M, 3), dtype=np.int32)
    for m in range(M):
        lib.or_mode_degrees(order, dim, basis, m, out[m].ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return out


def forcing_modes(dim, kmax):
    """Wave vectors of the driving field, (n, 3) int array (Sec. 7.1)."""
    lib = _load()
    n = lib.or_forcing_modes(dim, kmax, None)
    kv = np.zeros((n, 3), dtype=np.int32)
    lib.or_forcing_modes(dim, kmax, kv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return kv


def ou_update(dim, kv, amp, noise, dt, t_corr, sigma0):
    """One Ornstein-Uhlenbeck step of the amplitudes (nm, 3, 2); returns a copy."""
    lib = _load()
    kv = np.ascontiguousarray(kv, dtype=np.int32)
    a = np.array(amp, dtype=np.float64, order="C", copy=True)
    nz = np.ascontiguousarray(noise, dtype=np.float64)
    assert a.shape == (len(kv), 3, 2) and nz.shape == a.shape
    lib.or_ou_update(dim, len(kv), kv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(a), _ptr(nz),
                     float(dt), float(t_corr), float(sigma0))
    return a


def forcing_project(prob, lo, kv, amp):
    """DG coefficients (ncells, 3, p^d) of the driving field of the amplitudes."""
    lib = _load()
    kv = np.ascontiguousarray(kv, dtype=np.int32)
    a = np.ascontiguousarray(amp, dtype=np.float64)
    lo3 = np.zeros(3)
    lo3[:len(lo)] = lo
    out = np.zeros((prob.ncells, 3, prob.nmodes))
    lib.or_forcing_project(ctypes.byref(prob.p), _ptr(lo3), len(kv), kv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           _ptr(a), _ptr(out))
    return out


def legendre(lmax, x):
    lib = _load()
    P = np.zeros(lmax + 1)
    dP = np.zeros(lmax + 1)
    lib.or_legendre(lmax, float(x), _ptr(P), _ptr(dP))
    return P, dP


def gauss(n):
    lib = _load()
    x = np.zeros(n)
    w = np.zeros(n)
    lib.or_gauss(n, _ptr(x), _ptr(w))
    return x, w


def hllc(dim, gamma, uL, uR, axis):
    lib = _load()
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    F = np.zeros(dim + 2)
    lib.or_hllc(dim, gamma, _ptr(uL), _ptr(uR), axis, _ptr(F))
    return F


def euler_flux(dim, gamma, u, axis):
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.zeros(dim + 2)
    lib.or_euler_flux(dim, gamma, _ptr(u), axis, _ptr(f))
    return f


def sensor(order, dim, wrho):
    return _load().or_sensor(order, dim, _ptr(np.ascontiguousarray(wrho, dtype=np.float64)))


def sensor_rate(order, dim, wrho, wdrho):
    return _load().or_sensor_rate(order, dim, _ptr(np.ascontiguousarray(wrho, dtype=np.float64)),
                                  _ptr(np.ascontiguousarray(wdrho, dtype=np.float64)))


def rk_stages(order):
    return _load().or_rk_stages(order)


def recovery_fraction(order):
    return _load().or_recovery_fraction(order)


def num_threads():
    return _load().or_num_threads()


def set_num_threads(n):
    _load().or_set_num_threads(int(n))
