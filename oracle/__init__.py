"""CPU FP64 oracle for the APD hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The GPU library never loads it and shares
no code with it.

``apd_oracle.c`` holds the reference (brute-force Algorithm 1, the objective
(2.7) and gradient (2.8), L-BFGS for Algorithm 2, the Lloyd step of
Algorithm 3, the resolution rules (2.9)/(2.10)); this module is a ctypes
wrapper around it.  ``ref_numpy`` is an independent tiny NumPy brute force
used to cross-check the C code on small instances, and ``mlp`` is the FP64
reference of the warm-start network.

Instances are duck-typed: any object with ``dim, grid, lo, hi, x, A, v``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apd_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("grid", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("x", ctypes.c_void_p),
        ("A", ctypes.c_void_p),
        ("v", ctypes.c_void_p),
        ("mass", ctypes.c_void_p),
        ("power", ctypes.c_int32),
    ]


class _Opts(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("max_evals", ctypes.c_int32),
        ("history", ctypes.c_int32),
        ("gamma0", ctypes.c_double),
    ]


class _Report(ctypes.Structure):
    _fields_ = [
        ("converged", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("evals", ctypes.c_int32),
        ("f", ctypes.c_double),
        ("crit", ctypes.c_double),
    ]


_FG = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))

STATUS = {0: "ok", 4: "not_converged", 5: "linesearch"}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER(_Problem)
        vp = ctypes.c_void_p
        L.orc_pixel_volume.argtypes = [P]
        L.orc_pixel_volume.restype = ctypes.c_double
        L.orc_assign.argtypes = [P, vp, vp, vp, vp]
        L.orc_assign.restype = None
        L.orc_assign_pixels.argtypes = [P, vp, vp, ctypes.c_int64, vp, vp, vp]
        L.orc_assign_pixels.restype = None
        L.orc_evaluate.argtypes = [P, vp, vp, vp, vp, vp]
        L.orc_evaluate.restype = ctypes.c_double
        L.orc_two_loop.argtypes = [ctypes.c_int64, ctypes.c_int32, vp, vp, vp,
                                   ctypes.c_double, vp, vp]
        L.orc_two_loop.restype = None
        L.orc_lbfgs.argtypes = [ctypes.c_int64, vp, _FG, vp, ctypes.POINTER(_Opts),
                                ctypes.POINTER(_Report)]
        L.orc_lbfgs.restype = ctypes.c_int
        L.orc_default_gamma0.argtypes = [ctypes.c_int32, ctypes.c_int64]
        L.orc_default_gamma0.restype = ctypes.c_double
        L.orc_fit_weights.argtypes = [P, vp, ctypes.c_int32, ctypes.POINTER(_Opts),
                                      ctypes.POINTER(_Report)]
        L.orc_fit_weights.restype = ctypes.c_int
        L.orc_lloyd_step.argtypes = [P, vp, vp, ctypes.POINTER(_Opts), ctypes.POINTER(_Report)]
        L.orc_lloyd_step.restype = ctypes.c_int
        L.orc_fit_weights_refine.argtypes = [P, vp, ctypes.c_int32, ctypes.POINTER(_Opts),
                                             ctypes.c_int32, ctypes.POINTER(_Report), vp]
        L.orc_fit_weights_refine.restype = ctypes.c_int
        L.orc_domain_measure.argtypes = [P]
        L.orc_domain_measure.restype = ctypes.c_double
        L.orc_resolution_lower_bound.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double]
        L.orc_resolution_lower_bound.restype = ctypes.c_double
        L.orc_choose_resolution.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double]
        L.orc_choose_resolution.restype = ctypes.c_int64
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class _Bound:
    """Keeps the arrays referenced by a _Problem alive."""

    def __init__(self, inst, x=None):
        self.x = _f64(inst.x if x is None else x)
        self.A = _f64(inst.A)
        self.v = _f64(inst.v) if getattr(inst, "v", None) is not None else None
        m = getattr(inst, "mass", None)
        self.mass = np.ascontiguousarray(m, dtype=np.uint8).reshape(-1) if m is not None else None
        dim = int(inst.dim)
        p = _Problem()
        p.dim = dim
        p.n = self.x.shape[0]
        for d in range(3):
            p.grid[d] = int(inst.grid[d]) if d < dim else 1
            p.lo[d] = float(inst.lo[d]) if d < dim else 0.0
            p.hi[d] = float(inst.hi[d]) if d < dim else 1.0
        p.x = _ptr(self.x)
        p.A = _ptr(self.A)
        p.v = _ptr(self.v)
        p.mass = _ptr(self.mass)
        p.power = int(getattr(inst, "power", 2))
        self.p = p
        self.J = int(np.prod([int(g) for g in inst.grid]))
        if self.mass is not None and self.mass.size != self.J:
            raise ValueError("mass must hold one weight per pixel")

    def ref(self):
        return ctypes.byref(self.p)


def pixel_volume(inst) -> float:
    return lib().orc_pixel_volume(_Bound(inst).ref())


def pixel_centres(inst) -> np.ndarray:
    """(J, D) centres y_j, row-major, last axis fastest (eq. (2.6))."""
    axes = [inst.lo[d] + (np.arange(inst.grid[d], dtype=np.float64) + 0.5)
            * ((inst.hi[d] - inst.lo[d]) / inst.grid[d]) for d in range(inst.dim)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def assign(inst, w, x=None):
    """Algorithm 1: labels (int32, lowest index on ties), C_(1), C_(2)."""
    b = _Bound(inst, x)
    w = _f64(w)
    labels = np.empty(b.J, np.int32)
    best = np.empty(b.J, np.float64)
    second = np.empty(b.J, np.float64)
    lib().orc_assign(b.ref(), _ptr(w), _ptr(labels), _ptr(best), _ptr(second))
    return labels, best, second


def assign_pixels(inst, w, idx, x=None):
    """Algorithm 1 at the listed pixel indices: labels, C_(1), C_(2)."""
    b = _Bound(inst, x)
    w = _f64(w)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    labels = np.empty(len(idx), np.int32)
    best = np.empty(len(idx))
    second = np.empty(len(idx))
    lib().orc_assign_pixels(b.ref(), _ptr(w), _ptr(idx), len(idx), _ptr(labels), _ptr(best),
                            _ptr(second))
    return labels, best, second


@dataclass
class Evaluation:
    g: float
    grad: np.ndarray
    counts: np.ndarray
    centroids: np.ndarray
    maxrel: float


def evaluate(inst, w, x=None) -> Evaluation:
    """Objective (2.7), gradient (2.8), counts, centroids, max rel. error."""
    b = _Bound(inst, x)
    n = b.x.shape[0]
    w = _f64(w)
    grad = np.empty(n)
    counts = np.empty(n, np.int64)
    cen = np.empty((n, inst.dim))
    mr = ctypes.c_double()
    g = lib().orc_evaluate(b.ref(), _ptr(w), _ptr(grad), _ptr(counts), _ptr(cen),
                           ctypes.byref(mr))
    return Evaluation(g, grad, counts, cen, mr.value)


@dataclass
class Report:
    status: str
    converged: bool
    iters: int
    evals: int
    f: float
    crit: float


def _opts(eps, max_iter, max_evals, history, gamma0):
    o = _Opts()
    o.eps = eps
    o.max_iter = max_iter
    o.max_evals = max_evals
    o.history = history
    o.gamma0 = gamma0
    return o


def _report(st, r) -> Report:
    return Report(STATUS.get(st, str(st)), bool(r.converged), r.iters, r.evals, r.f, r.crit)


def default_gamma0(dim: int, n: int) -> float:
    return lib().orc_default_gamma0(dim, n)


def fit_weights(inst, w0=None, eps=0.01, max_iter=100000, max_evals=2000, history=10,
                gamma0=None, x=None):
    """Algorithm 2 (L-BFGS on -g~).  Returns (w, Report)."""
    b = _Bound(inst, x)
    n = b.x.shape[0]
    warm = w0 is not None
    w = _f64(np.zeros(n) if w0 is None else w0).copy()
    g0 = default_gamma0(inst.dim, n) if gamma0 is None else gamma0
    o = _opts(eps, max_iter, max_evals, history, g0)
    r = _Report()
    st = lib().orc_fit_weights(b.ref(), _ptr(w), int(warm), ctypes.byref(o), ctypes.byref(r))
    return w, _report(st, r)


def fit_weights_refine(inst, w0=None, eps=0.01, max_refine=3, max_iter=100000, max_evals=2000,
                       history=10, gamma0=None):
    """Algorithm 2 with its last step (refine the grid and restart when the
    tolerance is not reached).  Returns (w, Report, grid used)."""
    b = _Bound(inst)
    n = b.x.shape[0]
    warm = w0 is not None
    w = _f64(np.zeros(n) if w0 is None else w0).copy()
    g0 = default_gamma0(inst.dim, n) if gamma0 is None else gamma0
    o = _opts(eps, max_iter, max_evals, history, g0)
    r = _Report()
    grid = np.zeros(3, np.int32)
    st = lib().orc_fit_weights_refine(b.ref(), _ptr(w), int(warm), ctypes.byref(o), int(max_refine),
                                      ctypes.byref(r), _ptr(grid))
    return w, _report(st, r), tuple(int(g) for g in grid[:inst.dim])


def domain_measure(inst) -> float:
    """sum_j |P_j|: |Omega| without pixel weights."""
    return lib().orc_domain_measure(_Bound(inst).ref())


def lloyd_step(inst, x, w, eps=0.01, max_iter=100000, max_evals=2000, history=10,
               gamma0=None):
    """One loop pass of Algorithm 3: warm fit, then seeds -> discrete centroids.
    Returns (x_new, w_new, Report)."""
    b = _Bound(inst, x)
    n = b.x.shape[0]
    xx = b.x.copy()
    ww = _f64(w).copy()
    g0 = default_gamma0(inst.dim, n) if gamma0 is None else gamma0
    o = _opts(eps, max_iter, max_evals, history, g0)
    r = _Report()
    st = lib().orc_lloyd_step(b.ref(), _ptr(xx), _ptr(ww), ctypes.byref(o), ctypes.byref(r))
    return xx, ww, _report(st, r)


def lbfgs(fg, w0, eps, gamma0=1.0, max_iter=100000, max_evals=2000, history=10):
    """The solver on an arbitrary function: fg(w) -> (f, grad_f, crit)."""
    n = len(w0)
    w = _f64(w0).copy()
    errors = []

    def cb(_ctx, wp, gp, cp):
        try:
            ww = np.ctypeslib.as_array(wp, shape=(n,)).copy()
            f, gr, crit = fg(ww)
            ga = np.ctypeslib.as_array(gp, shape=(n,))
            ga[:] = gr
            cp[0] = crit
            return float(f)
        except Exception as e:  # pragma: no cover - surfaced below
            errors.append(e)
            cp[0] = 0.0
            return 0.0

    cfun = _FG(cb)
    o = _opts(eps, max_iter, max_evals, history, gamma0)
    r = _Report()
    st = lib().orc_lbfgs(n, _ptr(w), cfun, None, ctypes.byref(o), ctypes.byref(r))
    if errors:
        raise errors[0]
    return w, _report(st, r)


def two_loop(S, Y, gamma, q):
    """H q for the L-BFGS matrix built from pairs S[k], Y[k] (oldest first)."""
    S = _f64(S)
    Y = _f64(Y)
    q = _f64(q)
    npairs, n = S.shape
    rho = _f64(1.0 / np.einsum("ki,ki->k", S, Y))
    r = np.empty(n)
    lib().orc_two_loop(n, npairs, _ptr(S), _ptr(Y), _ptr(rho), float(gamma), _ptr(q), _ptr(r))
    return r


def resolution_lower_bound(dim: int, n: int, eps: float) -> float:
    """(N / eps)^(1/D), eq. (2.9)."""
    return lib().orc_resolution_lower_bound(dim, n, eps)


def choose_resolution(dim: int, eps: float, vmin: float, omega: float = 1.0) -> int:
    """Smallest M with |Omega| / M^D < eps / 2^D * min v, eq. (2.10)."""
    return int(lib().orc_choose_resolution(dim, eps, vmin, omega))


def num_threads() -> int:
    return int(lib().orc_num_threads())
