"""MI355X-native fitting of anisotropic power diagrams (arXiv 2403.03571).

A thin ctypes binding over ``libapd.so`` (the HIP library declared in
``include/apd.h``).  The functions keep the C names; they only marshal
torch tensors (device memory) and the current HIP stream into the C calls.
Every step of the computation runs in the library's kernels: there is no
CPU fallback, and loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapd.so")

APD_FP64, APD_FP32, APD_BF16 = 0, 1, 2
PRECISIONS = {"fp64": APD_FP64, "fp32": APD_FP32, "bf16": APD_BF16, "bf16-recheck": APD_BF16}

STATUS = {
    0: "APD_OK", 1: "APD_ERR_INVALID_ARG", 2: "APD_ERR_NOT_SPD", 3: "APD_ERR_VOLUMES",
    4: "APD_ERR_NOT_CONVERGED", 5: "APD_ERR_LINESEARCH", 6: "APD_ERR_DEVICE",
    7: "APD_ERR_OOM", 8: "APD_ERR_NONFINITE",
}


class ApdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class apd_problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("power", ctypes.c_int32), ("n", ctypes.c_int64),
        ("grid", ctypes.c_int32 * 3), ("reserved1", ctypes.c_int32),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("x", ctypes.c_void_p), ("A", ctypes.c_void_p), ("v", ctypes.c_void_p),
        ("mass", ctypes.c_void_p),
    ]


class apd_fit_opts(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double), ("max_iter", ctypes.c_int32), ("max_evals", ctypes.c_int32),
        ("history", ctypes.c_int32), ("warm", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("refine", ctypes.c_int32), ("gamma0", ctypes.c_double), ("coarse_eps", ctypes.c_double),
    ]


class apd_fit_report(ctypes.Structure):
    _fields_ = [
        ("converged", ctypes.c_int32), ("iters", ctypes.c_int32), ("evals", ctypes.c_int32),
        ("rechecked", ctypes.c_int32), ("max_rel_err", ctypes.c_double), ("g", ctypes.c_double),
        ("seconds", ctypes.c_double), ("grid", ctypes.c_int32 * 3), ("refinements", ctypes.c_int32),
        ("coarse_evals", ctypes.c_int32),
    ]


class apd_tune_result(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("culling", ctypes.c_int32),
                ("pixels_per_lane", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pass_ms", ctypes.c_double * 6)]


class apd_tune_batched_result(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("pixels_per_lane", ctypes.c_int32),
                ("fit_ms", ctypes.c_double * 6)]


# apd_kernel
KERNELS = {"fp32-matrix": 0, "fp32-vector": 1, "fp32-lists": 2, "bf16-matrix": 3, "bf16-lists": 4, "fp64": 5,
           "fp32-hybrid": 6}
KERNEL_NAMES = {v: k for k, v in KERNELS.items()}


class apd_pass_stats(ctypes.Structure):
    _fields_ = [("pixels", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("rechecked", ctypes.c_int64), ("assign_ms", ctypes.c_double),
                ("pass_ms", ctypes.c_double), ("tiles_credited", ctypes.c_int64),
                ("kernel", ctypes.c_int32), ("pixels_per_lane", ctypes.c_int32)]


# every symbol include/apd.h declares
EXPORTS = [
    "apd_create", "apd_destroy", "apd_last_error", "apd_set_stream", "apd_assign",
    "apd_dual_objective_grad", "apd_fit_weights", "apd_lloyd_step", "apd_choose_resolution",
    "apd_last_pass_stats", "apd_set_profiling", "apd_set_variant", "apd_fit_weights_batched",
    "apd_ws_create", "apd_ws_destroy", "apd_ws_get_params", "apd_ws_features", "apd_ws_forward",
    "apd_ws_infer",
    "apd_ws_loss_grad", "apd_ws_train_step", "apd_ws_predict", "apd_fit_weights_ws",
    "apd_ws_targets", "apd_set_culling", "apd_autotune", "apd_set_pixels_per_lane",
    "apd_measure_valu_rate", "apd_set_adaptive", "apd_dual_objective_grad_noalloc",
    "apd_autotune_batched", "apd_set_batch_kernel", "apd_ws_train_epoch",
]

WS_PARAMS = 35841  # 20*128 + 128 + 2*(128*128 + 128) + 128 + 1
WS_FEATURES = 20

_lib = None
_live = []  # weak references to every open context / network


def _close_all():
    # release device objects before the HIP runtime is torn down at exit
    for ref in reversed(_live):
        obj = ref()
        if obj is not None:
            try:
                obj.close()
            except Exception:
                pass
    _live.clear()


import atexit as _atexit  # noqa: E402
import weakref as _weakref  # noqa: E402

_atexit.register(_close_all)


def lib():
    """Load libapd.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER(apd_problem)
    L.apd_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    L.apd_create.restype = ctypes.c_int
    L.apd_destroy.argtypes = [vp]
    L.apd_destroy.restype = None
    L.apd_last_error.argtypes = [vp]
    L.apd_last_error.restype = ctypes.c_char_p
    L.apd_set_stream.argtypes = [vp, vp]
    L.apd_set_stream.restype = ctypes.c_int
    L.apd_assign.argtypes = [vp, P, vp, vp, vp, ctypes.c_int]
    L.apd_assign.restype = ctypes.c_int
    L.apd_dual_objective_grad.argtypes = [vp, P, vp, ctypes.POINTER(dbl), vp, vp, vp,
                                          ctypes.POINTER(dbl), ctypes.c_int]
    L.apd_dual_objective_grad.restype = ctypes.c_int
    L.apd_dual_objective_grad_noalloc.argtypes = L.apd_dual_objective_grad.argtypes
    L.apd_dual_objective_grad_noalloc.restype = ctypes.c_int
    L.apd_fit_weights.argtypes = [vp, P, vp, ctypes.POINTER(apd_fit_opts),
                                  ctypes.POINTER(apd_fit_report)]
    L.apd_fit_weights.restype = ctypes.c_int
    L.apd_lloyd_step.argtypes = [vp, P, vp, vp, ctypes.POINTER(apd_fit_opts),
                                 ctypes.POINTER(apd_fit_report)]
    L.apd_lloyd_step.restype = ctypes.c_int
    L.apd_choose_resolution.argtypes = [i32, dbl, dbl, dbl, ctypes.POINTER(i32)]
    L.apd_choose_resolution.restype = ctypes.c_int
    L.apd_last_pass_stats.argtypes = [vp, ctypes.POINTER(apd_pass_stats)]
    L.apd_last_pass_stats.restype = ctypes.c_int
    L.apd_set_profiling.argtypes = [vp, i32]
    L.apd_set_profiling.restype = ctypes.c_int
    L.apd_set_variant.argtypes = [vp, i32]
    L.apd_set_variant.restype = ctypes.c_int
    L.apd_fit_weights_batched.argtypes = [vp, P, i32, ctypes.POINTER(vp),
                                          ctypes.POINTER(apd_fit_opts), ctypes.POINTER(apd_fit_report)]
    L.apd_fit_weights_batched.restype = ctypes.c_int
    L.apd_ws_create.argtypes = [vp, ctypes.POINTER(vp), vp, i64]
    L.apd_ws_create.restype = ctypes.c_int
    L.apd_ws_destroy.argtypes = [vp]
    L.apd_ws_destroy.restype = None
    L.apd_ws_get_params.argtypes = [vp, vp, vp, i64]
    L.apd_ws_get_params.restype = ctypes.c_int
    L.apd_ws_features.argtypes = [vp, P, vp]
    L.apd_ws_features.restype = ctypes.c_int
    L.apd_ws_forward.argtypes = [vp, vp, vp, i64, vp]
    L.apd_ws_forward.restype = ctypes.c_int
    L.apd_ws_infer.argtypes = [vp, vp, vp, i64, vp]
    L.apd_ws_infer.restype = ctypes.c_int
    L.apd_ws_loss_grad.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(dbl), vp]
    L.apd_ws_loss_grad.restype = ctypes.c_int
    L.apd_ws_train_step.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.POINTER(dbl)]
    L.apd_ws_train_step.restype = ctypes.c_int
    L.apd_ws_train_epoch.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.POINTER(dbl)]
    L.apd_ws_train_epoch.restype = ctypes.c_int
    L.apd_ws_predict.argtypes = [vp, vp, P, vp]
    L.apd_ws_predict.restype = ctypes.c_int
    L.apd_fit_weights_ws.argtypes = [vp, vp, P, vp, ctypes.POINTER(apd_fit_opts),
                                     ctypes.POINTER(apd_fit_report), ctypes.POINTER(i32)]
    L.apd_fit_weights_ws.restype = ctypes.c_int
    L.apd_ws_targets.argtypes = [vp, i64, vp, vp]
    L.apd_ws_targets.restype = ctypes.c_int
    L.apd_set_culling.argtypes = [vp, i32]
    L.apd_set_culling.restype = ctypes.c_int
    L.apd_set_adaptive.argtypes = [vp, i32]
    L.apd_set_adaptive.restype = ctypes.c_int
    L.apd_set_pixels_per_lane.argtypes = [vp, i32]
    L.apd_set_pixels_per_lane.restype = ctypes.c_int
    L.apd_autotune.argtypes = [vp, P, vp, ctypes.c_int, i32, ctypes.POINTER(apd_tune_result)]
    L.apd_autotune.restype = ctypes.c_int
    L.apd_autotune_batched.argtypes = [vp, P, i32, i32, ctypes.POINTER(apd_tune_batched_result)]
    L.apd_autotune_batched.restype = ctypes.c_int
    L.apd_set_batch_kernel.argtypes = [vp, i32, i32]
    L.apd_set_batch_kernel.restype = ctypes.c_int
    L.apd_measure_valu_rate.argtypes = [i32, i32, ctypes.POINTER(dbl)]
    L.apd_measure_valu_rate.restype = ctypes.c_int
    _lib = L
    return L


def _torch():
    import torch
    return torch


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _check_dev(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """Device-resident APD problem: seeds x (n, D), matrices A (n, D, D),
    volumes v (n,) as float64 tensors, plus the box and the grid."""

    def __init__(self, dim, grid, lo, hi, x, A, v=None, mass=None, power=2):
        self.dim = int(dim)
        self.power = int(power)   # cost |y - x|_A^power - w
        self.grid = tuple(int(g) for g in grid)
        self.lo = tuple(float(t) for t in lo)
        self.hi = tuple(float(t) for t in hi)
        self.x, self.A, self.v = x, A, v
        self.mass = mass   # optional uint8 pixel weights (J,)
        self.n = int(x.shape[0])
        self.J = int(np.prod(self.grid))

    @classmethod
    def from_instance(cls, inst, device="cuda"):
        torch = _torch()
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64), device=device)
        m = getattr(inst, "mass", None)
        mass = None if m is None else torch.as_tensor(np.ascontiguousarray(m, np.uint8).reshape(-1),
                                                     device=device)
        return cls(inst.dim, inst.grid, inst.lo, inst.hi, f(inst.x), f(inst.A),
                   None if inst.v is None else f(inst.v), mass, int(getattr(inst, "power", 2)))

    def c_struct(self, x=None) -> apd_problem:
        torch = _torch()
        p = apd_problem()
        p.dim, p.n = self.dim, self.n
        p.power = self.power
        for d in range(3):
            p.grid[d] = self.grid[d] if d < self.dim else 1
            p.lo[d] = self.lo[d] if d < self.dim else 0.0
            p.hi[d] = self.hi[d] if d < self.dim else 1.0
        xx = self.x if x is None else x
        p.x = _check_dev(xx, torch.float64, (self.n, self.dim), "x").value
        p.A = _check_dev(self.A, torch.float64, (self.n, self.dim, self.dim), "A").value
        p.v = (_check_dev(self.v, torch.float64, (self.n,), "v").value
               if self.v is not None else None)
        p.mass = (_check_dev(self.mass, torch.uint8, (self.J,), "mass").value
                  if self.mass is not None else None)
        return p


@dataclass
class FitReport:
    status: str
    converged: bool
    iters: int
    evals: int
    rechecked: int
    max_rel_err: float
    g: float
    seconds: float
    grid: tuple = ()
    refinements: int = 0
    coarse_evals: int = 0


class Context:
    """An apd_ctx on one device.  Calls enqueue on torch's current stream."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.device = int(device)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib().apd_create(ctypes.byref(self._h), self.device,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        if st != 0:
            raise ApdError(st, "apd_create failed")
        _live.append(_weakref.ref(self))

    def close(self):
        if self._h:
            lib().apd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        torch = _torch()
        lib().apd_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _raise(self, st):
        if st != 0:
            raise ApdError(st, lib().apd_last_error(self._h).decode())

    # --- the C calls -----------------------------------------------------
    def apd_assign(self, prob: Problem, w, labels=None, prec="fp32", rel_gap=False):
        """Algorithm 1: labels (J,) int32; with ``rel_gap`` also the (J,)
        float32 lower bounds of the relative top-two gaps, as (labels, gap)."""
        torch = _torch()
        self._stream()
        if labels is None:
            labels = torch.empty(prob.J, dtype=torch.int32, device=w.device)
        p = prob.c_struct()
        wp = _check_dev(w, torch.float64, (prob.n,), "w")
        lp = _check_dev(labels, torch.int32, (prob.J,), "labels")
        gap = None
        if rel_gap is not False and rel_gap is not None:
            gap = (torch.empty(prob.J, dtype=torch.float32, device=w.device) if rel_gap is True
                   else rel_gap)
            gp = _check_dev(gap, torch.float32, (prob.J,), "rel_gap")
        else:
            gp = None
        self._raise(lib().apd_assign(self._h, ctypes.byref(p), wp, lp, gp, _prec(prec)))
        return labels if gap is None else (labels, gap)

    def apd_dual_objective_grad(self, prob: Problem, w, prec="fp32", counts=False,
                                centroids=False, x=None, grad=None, noalloc=False):
        """eq. (2.7) and its gradient (2.8) at w.  ``grad``: an optional
        output tensor (n,) float64 on the device (else one is allocated).
        ``noalloc``: call apd_dual_objective_grad_noalloc (the library's
        scratch in its static array; the outputs are still allocated here
        unless passed in)."""
        torch = _torch()
        self._stream()
        p = prob.c_struct(x)
        dev = w.device
        if grad is None:
            grad = torch.empty(prob.n, dtype=torch.float64, device=dev)
        else:
            _check_dev(grad, torch.float64, (prob.n,), "grad")
        cnt = torch.empty(prob.n, dtype=torch.int64, device=dev) if counts else None
        cen = torch.empty((prob.n, prob.dim), dtype=torch.float64, device=dev) if centroids else None
        g = ctypes.c_double()
        mr = ctypes.c_double()
        wp = _check_dev(w, torch.float64, (prob.n,), "w")
        call = lib().apd_dual_objective_grad_noalloc if noalloc else lib().apd_dual_objective_grad
        st = call(
            self._h, ctypes.byref(p), wp, ctypes.byref(g), ctypes.c_void_p(grad.data_ptr()),
            ctypes.c_void_p(cnt.data_ptr()) if cnt is not None else None,
            ctypes.c_void_p(cen.data_ptr()) if cen is not None else None,
            ctypes.byref(mr), _prec(prec))
        self._raise(st)
        out = {"g": g.value, "grad": grad, "maxrel": mr.value}
        if cnt is not None:
            out["counts"] = cnt
        if cen is not None:
            out["centroids"] = cen
        return out

    @staticmethod
    def _opts(eps, max_iter, max_evals, history, warm, prec, gamma0, refine=0, coarse_eps=0.0):
        o = apd_fit_opts()
        o.eps, o.max_iter, o.max_evals, o.history = eps, max_iter, max_evals, history
        o.warm, o.prec, o.gamma0, o.refine = int(warm), _prec(prec), gamma0, int(refine)
        o.coarse_eps = float(coarse_eps)
        return o

    @staticmethod
    def _report(st, r) -> FitReport:
        return FitReport(STATUS.get(st, str(st)), bool(r.converged), r.iters, r.evals,
                         r.rechecked, r.max_rel_err, r.g, r.seconds, tuple(r.grid),
                         int(r.refinements), int(r.coarse_evals))

    def apd_fit_weights(self, prob: Problem, w=None, eps=0.01, max_iter=100000, max_evals=2000,
                        history=10, prec="fp32", gamma0=0.0, raise_on_fail=False, refine=0,
                        coarse_eps=0.0):
        torch = _torch()
        self._stream()
        warm = w is not None
        if w is None:
            w = torch.zeros(prob.n, dtype=torch.float64, device=prob.x.device)
        p = prob.c_struct()
        o = self._opts(eps, max_iter, max_evals, history, warm, prec, gamma0, refine, coarse_eps)
        r = apd_fit_report()
        wp = _check_dev(w, torch.float64, (prob.n,), "w")
        st = lib().apd_fit_weights(self._h, ctypes.byref(p), wp, ctypes.byref(o), ctypes.byref(r))
        if st not in (0, 4, 5) or (raise_on_fail and st != 0):
            self._raise(st)
        return w, self._report(st, r)

    def apd_fit_weights_batched(self, probs, ws=None, eps=0.01, max_iter=100000, max_evals=2000,
                                history=10, prec="fp32", gamma0=0.0):
        """Algorithm 2 for every problem of `probs` in one batched solve.
        Returns (list of w tensors, list of FitReport, status)."""
        torch = _torch()
        self._stream()
        B = len(probs)
        warm = ws is not None
        if ws is None:
            ws = [torch.zeros(p.n, dtype=torch.float64, device=p.x.device) for p in probs]
        arr = (apd_problem * B)(*[p.c_struct() for p in probs])
        ptrs = (ctypes.c_void_p * B)(*[_check_dev(w, torch.float64, (p.n,), "w").value
                                        for w, p in zip(ws, probs)])
        o = self._opts(eps, max_iter, max_evals, history, warm, prec, gamma0)
        reps = (apd_fit_report * B)()
        st = lib().apd_fit_weights_batched(self._h, arr, B, ptrs, ctypes.byref(o), reps)
        if st not in (0, 4):
            self._raise(st)
        return ws, [self._report(0 if r.converged else 4, r) for r in reps], STATUS.get(st, st)

    def apd_lloyd_step(self, prob: Problem, x, w, eps=0.01, max_iter=100000, max_evals=2000,
                       history=10, prec="fp32", gamma0=0.0):
        torch = _torch()
        self._stream()
        p = prob.c_struct(x)
        o = self._opts(eps, max_iter, max_evals, history, True, prec, gamma0)
        r = apd_fit_report()
        xp = _check_dev(x, torch.float64, (prob.n, prob.dim), "x")
        wp = _check_dev(w, torch.float64, (prob.n,), "w")
        st = lib().apd_lloyd_step(self._h, ctypes.byref(p), xp, wp, ctypes.byref(o), ctypes.byref(r))
        if st not in (0, 4, 5):
            self._raise(st)
        return x, w, self._report(st, r)

    def apd_last_pass_stats(self):
        s = apd_pass_stats()
        self._raise(lib().apd_last_pass_stats(self._h, ctypes.byref(s)))
        return {"pixels": s.pixels, "pairs": s.pairs, "rechecked": s.rechecked,
                "assign_ms": s.assign_ms, "pass_ms": s.pass_ms, "tiles_credited": s.tiles_credited,
                "kernel": KERNEL_NAMES.get(s.kernel, s.kernel), "pixels_per_lane": s.pixels_per_lane}

    def apd_set_profiling(self, on: bool):
        self._raise(lib().apd_set_profiling(self._h, int(bool(on))))

    def apd_autotune(self, prob: Problem, w=None, prec="fp32", reps=5):
        """Time the exact kernels of the tier on prob, keep the fastest.
        Returns {"variant", "culling", "pixels_per_lane",
        "pass_ms": [cull P4, cull P8, full P4, full P8, matrix, hybrid]}."""
        torch = _torch()
        self._stream()
        if w is None:
            w = torch.zeros(prob.n, dtype=torch.float64, device=prob.x.device)
        p = prob.c_struct()
        r = apd_tune_result()
        wp = _check_dev(w, torch.float64, (prob.n,), "w")
        self._raise(lib().apd_autotune(self._h, ctypes.byref(p), wp, _prec(prec), int(reps),
                                       ctypes.byref(r)))
        return {"variant": r.variant, "culling": r.culling, "pixels_per_lane": r.pixels_per_lane,
                "pass_ms": list(r.pass_ms)}

    def apd_autotune_batched(self, probs, evals=8):
        """Time every batched kernel on the solve of probs (evals evaluations
        per instance from W_0 = 0) and keep the fastest for
        apd_fit_weights_batched.  Returns {"kernel", "pixels_per_lane",
        "fit_ms": [lists P4, lists P8, vector, fp32 matrix, bf16 lists,
        bf16 matrix]}."""
        self._stream()
        B = len(probs)
        arr = (apd_problem * B)(*[p.c_struct() for p in probs])
        r = apd_tune_batched_result()
        self._raise(lib().apd_autotune_batched(self._h, arr, B, int(evals), ctypes.byref(r)))
        return {"kernel": KERNEL_NAMES[r.kernel], "pixels_per_lane": r.pixels_per_lane,
                "fit_ms": list(r.fit_ms)}

    def apd_set_batch_kernel(self, kernel, pixels_per_lane=0):
        """Kernel of apd_fit_weights_batched: None (by tier) or a KERNELS name."""
        k = -1 if kernel is None else KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        self._raise(lib().apd_set_batch_kernel(self._h, k, int(pixels_per_lane)))

    def apd_set_pixels_per_lane(self, p: int):
        self._raise(lib().apd_set_pixels_per_lane(self._h, int(p)))

    def apd_set_adaptive(self, on: bool):
        self._raise(lib().apd_set_adaptive(self._h, int(bool(on))))

    def apd_set_culling(self, on: bool):
        """Per-tile candidate lists in the vector APD_FP32 kernel."""
        self._raise(lib().apd_set_culling(self._h, int(bool(on))))

    def apd_set_variant(self, variant: int):
        """APD_FP32 kernel: 0 = matrix cores, 1 = vector ALU."""
        self._raise(lib().apd_set_variant(self._h, int(variant)))


def apd_measure_valu_rate(device: int = 0, op: str = "fma") -> float:
    """Sustained vector-ALU lane operations per second (op "fma" or "add")."""
    out = ctypes.c_double(0.0)
    st = lib().apd_measure_valu_rate(int(device), {"fma": 0, "add": 1}[op], ctypes.byref(out))
    if st != 0:
        raise ApdError(st, "apd_measure_valu_rate failed")
    return out.value


def apd_choose_resolution(dim: int, eps: float, vmin: float, omega: float = 1.0) -> int:
    M = ctypes.c_int32()
    st = lib().apd_choose_resolution(dim, eps, vmin, omega, ctypes.byref(M))
    if st != 0:
        raise ApdError(st, "apd_choose_resolution: invalid argument")
    return int(M.value)


class WarmStart:
    """The learned warm start (an apd_ws_model): a per-seed network whose
    parameters live on the device.  `params` is the initial flat float32
    vector (its random draws are the caller's)."""

    def __init__(self, ctx: Context, params):
        self.ctx = ctx
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != WS_PARAMS:
            raise ValueError(f"the network has {WS_PARAMS} parameters")
        self._h = ctypes.c_void_p()
        ctx._stream()
        ctx._raise(lib().apd_ws_create(ctx._h, ctypes.byref(self._h),
                                       p.ctypes.data_as(ctypes.c_void_p), p.size))
        _live.append(_weakref.ref(self))

    def close(self):
        if self._h:
            lib().apd_ws_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(WS_PARAMS, np.float32)
        self.ctx._raise(lib().apd_ws_get_params(self.ctx._h, self._h,
                                                out.ctypes.data_as(ctypes.c_void_p), out.size))
        return out

    def features(self, prob: Problem):
        torch = _torch()
        self.ctx._stream()
        F = torch.empty((prob.n, WS_FEATURES), dtype=torch.float32, device=prob.x.device)
        p = prob.c_struct()
        self.ctx._raise(lib().apd_ws_features(self.ctx._h, ctypes.byref(p),
                                              ctypes.c_void_p(F.data_ptr())))
        return F

    def targets(self, w):
        """t = N (w - mean w) of solver weights w (float32 tensor)."""
        torch = _torch()
        self.ctx._stream()
        n = int(w.shape[0])
        wp = _check_dev(w, torch.float64, (n,), "w")
        t = torch.empty(n, dtype=torch.float32, device=w.device)
        self.ctx._raise(lib().apd_ws_targets(self.ctx._h, n, wp, ctypes.c_void_p(t.data_ptr())))
        return t

    def forward(self, F):
        torch = _torch()
        self.ctx._stream()
        S = int(F.shape[0])
        Fp = _check_dev(F, torch.float32, (S, WS_FEATURES), "F")
        y = torch.empty(S, dtype=torch.float32, device=F.device)
        self.ctx._raise(lib().apd_ws_forward(self.ctx._h, self._h, Fp, S,
                                             ctypes.c_void_p(y.data_ptr())))
        return y

    def infer(self, F):
        """The network output for inference: BF16 matrix-core operands, FP32
        accumulation (what predict uses)."""
        torch = _torch()
        self.ctx._stream()
        S = int(F.shape[0])
        Fp = _check_dev(F, torch.float32, (S, WS_FEATURES), "F")
        y = torch.empty(S, dtype=torch.float32, device=F.device)
        self.ctx._raise(lib().apd_ws_infer(self.ctx._h, self._h, Fp, S,
                                           ctypes.c_void_p(y.data_ptr())))
        return y

    def loss_grad(self, F, t):
        torch = _torch()
        self.ctx._stream()
        S = int(F.shape[0])
        Fp = _check_dev(F, torch.float32, (S, WS_FEATURES), "F")
        tp = _check_dev(t, torch.float32, (S,), "t")
        g = torch.empty(WS_PARAMS, dtype=torch.float32, device=F.device)
        loss = ctypes.c_double()
        self.ctx._raise(lib().apd_ws_loss_grad(self.ctx._h, self._h, Fp, tp, S, ctypes.byref(loss),
                                               ctypes.c_void_p(g.data_ptr())))
        return loss.value, g

    def train_step(self, F, t, lr: float) -> float:
        torch = _torch()
        self.ctx._stream()
        S = int(F.shape[0])
        Fp = _check_dev(F, torch.float32, (S, WS_FEATURES), "F")
        tp = _check_dev(t, torch.float32, (S,), "t")
        loss = ctypes.c_double()
        self.ctx._raise(lib().apd_ws_train_step(self.ctx._h, self._h, Fp, tp, S, float(lr),
                                                ctypes.byref(loss)))
        return loss.value

    def train_epoch(self, F, t, lr: float) -> float:
        """apd_ws_train_epoch: Adam steps over minibatches of 4096 consecutive
        samples; returns the sample-weighted mean minibatch loss."""
        torch = _torch()
        self.ctx._stream()
        S = int(F.shape[0])
        Fp = _check_dev(F, torch.float32, (S, WS_FEATURES), "F")
        tp = _check_dev(t, torch.float32, (S,), "t")
        loss = ctypes.c_double()
        self.ctx._raise(lib().apd_ws_train_epoch(self.ctx._h, self._h, Fp, tp, S, float(lr),
                                                 ctypes.byref(loss)))
        return loss.value

    def predict(self, prob: Problem):
        torch = _torch()
        self.ctx._stream()
        w = torch.empty(prob.n, dtype=torch.float64, device=prob.x.device)
        p = prob.c_struct()
        self.ctx._raise(lib().apd_ws_predict(self.ctx._h, self._h, ctypes.byref(p),
                                             ctypes.c_void_p(w.data_ptr())))
        return w

    def fit(self, prob: Problem, eps=0.01, max_iter=100000, max_evals=2000, history=10,
            prec="fp32", gamma0=0.0):
        """Predict, fit warm, fall back to the cold start if needed.
        Returns (w, FitReport, used_warm)."""
        torch = _torch()
        self.ctx._stream()
        w = torch.empty(prob.n, dtype=torch.float64, device=prob.x.device)
        p = prob.c_struct()
        o = Context._opts(eps, max_iter, max_evals, history, True, prec, gamma0)
        r = apd_fit_report()
        used = ctypes.c_int32()
        st = lib().apd_fit_weights_ws(self.ctx._h, self._h, ctypes.byref(p),
                                      ctypes.c_void_p(w.data_ptr()), ctypes.byref(o),
                                      ctypes.byref(r), ctypes.byref(used))
        if st not in (0, 4, 5):
            self.ctx._raise(st)
        return w, Context._report(st, r), bool(used.value)
