"""MI355X (gfx950) RPY-FMM: Python binding of the C ABI in include/rpyfmm.h.

Argument marshalling only: every step of the matvec runs in the HIP kernels of
``librpyfmm.so``; PyTorch provides device memory and the stream.  The module
fails loudly if the library has not been built (``python -m
paper_1711_02976_amd.build``) -- there is no CPU fallback.

Functions mirror the C entry points (``rpy_plan``, ``rpy_plan_batched``,
``rpy_matvec``, ``rpy_sqrt_matvec``, ``rpy_plan_stats``, ``rpy_plan_export``,
``rpy_plan_free``); ``Plan`` wraps them for torch tensors::

    import torch, paper_1711_02976_amd as R
    pos = torch.rand(100_000, 3, dtype=torch.float64, device="cuda") * 50
    P = R.Plan(pos, a=0.5, eta=1.0, eps=1e-6, precision="mixed", nrhs=1)
    u = P.matvec(torch.randn(1, 100_000, 3, dtype=torch.float64, device="cuda"))
    y, info = P.sqrt_matvec(torch.randn_like(u), tol=1e-3)   # D^{1/2} z
    P.free()
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpyfmm.so")

RPY_OK, RPY_EINVAL, RPY_ENONFINITE, RPY_ENOMEM, RPY_EDEVICE, RPY_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RPY_INJECT_ALLOC = 100  # rpy_plan_inject_error: fail the next matvec-workspace allocation
PREC_FP64, PREC_MIXED = 0, 1
LIST_NAMES = ("U", "V", "W", "X", "O")


class rpy_options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("precision", C.c_int32), ("leaf_size", C.c_int32),
                ("order", C.c_int32), ("max_depth", C.c_int32), ("m2l_mode", C.c_int32),
                ("stream", C.c_void_p), ("nrhs", C.c_int32), ("w_direct", C.c_int32), ("eval_mode", C.c_int32), ("tune", C.c_int32)]


class rpy_plan_stats_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("nsys", C.c_int32), ("order", C.c_int32), ("leaf_size", C.c_int32),
                ("depth", C.c_int32), ("precision", C.c_int32), ("m2l_mode", C.c_int32),
                ("nbox", C.c_int64), ("nleaf", C.c_int64), ("list_len", C.c_int64 * 5),
                ("device_bytes", C.c_int64), ("plan_ms", C.c_double), ("w_direct", C.c_int32),
                ("p2l_items", C.c_int32), ("p2l_split_boxes", C.c_int32), ("sort_passes", C.c_int32),
                ("bead_pass_ms", C.c_double), ("eval_mode", C.c_int32), ("tuned", C.c_int32),
                ("tune_err", C.c_double)]


PHASES = ("permute", "p2p", "overlap", "p2m", "m2m", "m2l", "p2l", "l2l", "eval", "unpermute")


class rpy_timings_t(C.Structure):
    _fields_ = [("ms", C.c_double * len(PHASES)), ("launches", C.c_int64 * len(PHASES)), ("passes", C.c_int64),
                ("p2p_mc_ms", C.c_double), ("p2p_mc_launches", C.c_int64),
                ("p2p_mc_rhs", C.c_int64)]


class rpy_sqrt_info_t(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_change", C.c_double),
                ("min_ritz", C.c_double)]


class RpyError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None

EXPORTED = ("rpy_default_options", "rpy_plan", "rpy_plan_batched", "rpy_matvec", "rpy_matvec_noalloc",
            "rpy_sqrt_matvec", "rpy_plan_stats",
            "rpy_plan_export", "rpy_plan_set_timing", "rpy_plan_timings", "rpy_plan_inject_error", "rpy_plan_free",
            "rpy_status_string", "rpy_last_error")


def lib():
    """Load librpyfmm.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1711_02976_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.rpy_default_options.argtypes = [C.POINTER(rpy_options)]
        L.rpy_plan.argtypes = [C.POINTER(C.c_void_p), C.c_int64, C.c_void_p, C.c_double, C.c_double,
                               C.c_double, C.POINTER(rpy_options)]
        L.rpy_plan.restype = C.c_int
        L.rpy_plan_batched.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_int64), C.c_void_p,
                                       C.c_double, C.c_double, C.c_double, C.POINTER(rpy_options)]
        L.rpy_plan_batched.restype = C.c_int
        L.rpy_matvec.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.rpy_matvec.restype = C.c_int
        L.rpy_matvec_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.rpy_matvec_noalloc.restype = C.c_int
        L.rpy_sqrt_matvec.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                      C.POINTER(rpy_sqrt_info_t)]
        L.rpy_sqrt_matvec.restype = C.c_int
        L.rpy_plan_stats.argtypes = [C.c_void_p, C.POINTER(rpy_plan_stats_t)]
        L.rpy_plan_stats.restype = C.c_int
        L.rpy_plan_export.argtypes = [C.c_void_p] + [C.c_void_p] * 5
        L.rpy_plan_export.restype = C.c_int
        L.rpy_plan_set_timing.argtypes = [C.c_void_p, C.c_int32]
        L.rpy_plan_set_timing.restype = C.c_int
        L.rpy_plan_timings.argtypes = [C.c_void_p, C.POINTER(rpy_timings_t)]
        L.rpy_plan_timings.restype = C.c_int
        L.rpy_plan_inject_error.argtypes = [C.c_void_p, C.c_int32]
        L.rpy_plan_inject_error.restype = C.c_int
        L.rpy_plan_free.argtypes = [C.c_void_p]
        L.rpy_status_string.argtypes = [C.c_int]
        L.rpy_status_string.restype = C.c_char_p
        L.rpy_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != RPY_OK:
        L = lib()
        raise RpyError(status, f"{L.rpy_status_string(status).decode()}: {L.rpy_last_error().decode()}")


M2L_MODES = {"auto": 0, "dense": 1, "rotation": 2}


EVAL_MODES = {"auto": 0, "sets": 1, "poly": 2}


def make_options(precision=PREC_FP64, leaf_size=0, order=0, max_depth=0, stream=None, m2l="auto", nrhs=0,
                 w_direct=0, eval_mode="auto", tune=0):
    o = rpy_options()
    lib().rpy_default_options(C.byref(o))
    o.m2l_mode = M2L_MODES[m2l] if isinstance(m2l, str) else int(m2l)
    o.precision = int(precision)
    o.leaf_size = int(leaf_size)
    o.order = int(order)
    o.max_depth = int(max_depth)
    o.stream = stream
    o.nrhs = int(nrhs)
    o.w_direct = int(w_direct)
    o.eval_mode = EVAL_MODES[eval_mode] if isinstance(eval_mode, str) else int(eval_mode)
    o.tune = int(tune)
    return o


# ---- thin wrappers with the C names --------------------------------------
def rpy_plan(n, positions_ptr, a, eta, eps, options=None):
    h = C.c_void_p()
    st = lib().rpy_plan(C.byref(h), int(n), positions_ptr, float(a), float(eta), float(eps),
                        C.byref(options) if options is not None else None)
    _check(st)
    return h


def rpy_plan_batched(counts, positions_ptr, a, eta, eps, options=None):
    arr = (C.c_int64 * len(counts))(*[int(c) for c in counts])
    h = C.c_void_p()
    st = lib().rpy_plan_batched(C.byref(h), len(counts), arr, positions_ptr, float(a), float(eta), float(eps),
                                C.byref(options) if options is not None else None)
    _check(st)
    return h


def rpy_matvec(plan, nrhs, forces_ptr, velocities_ptr):
    _check(lib().rpy_matvec(plan, int(nrhs), forces_ptr, velocities_ptr))


def rpy_matvec_noalloc(plan, nrhs, forces_ptr, velocities_ptr):
    _check(lib().rpy_matvec_noalloc(plan, int(nrhs), forces_ptr, velocities_ptr))


def rpy_sqrt_matvec(plan, nrhs, z_ptr, y_ptr, tol, max_iter):
    info = rpy_sqrt_info_t()
    _check(lib().rpy_sqrt_matvec(plan, int(nrhs), z_ptr, y_ptr, float(tol), int(max_iter), C.byref(info)))
    return {"iterations": info.iterations, "converged": bool(info.converged), "rel_change": info.rel_change,
            "min_ritz": info.min_ritz}


def rpy_plan_stats(plan):
    s = rpy_plan_stats_t()
    _check(lib().rpy_plan_stats(plan, C.byref(s)))
    return {"n": s.n, "nsys": s.nsys, "order": s.order, "leaf_size": s.leaf_size, "depth": s.depth,
            "precision": s.precision, "m2l_mode": s.m2l_mode, "nbox": s.nbox, "nleaf": s.nleaf,
            "list_len": dict(zip(LIST_NAMES, list(s.list_len))), "device_bytes": s.device_bytes,
            "plan_ms": s.plan_ms, "w_direct": s.w_direct, "p2l_items": s.p2l_items,
            "p2l_split_boxes": s.p2l_split_boxes, "sort_passes": s.sort_passes, "bead_pass_ms": s.bead_pass_ms,
            "eval_mode": {1: "sets", 2: "poly"}.get(s.eval_mode, s.eval_mode),
            "tuned": {0: "model", 1: "measured", 2: "cached"}.get(s.tuned, s.tuned), "tune_err": s.tune_err}


def rpy_plan_export(plan):
    st = rpy_plan_stats(plan)
    n, nbox = st["n"], st["nbox"]
    perm = np.zeros(max(n, 1), dtype=np.int64)
    keys = np.zeros(max(n, 1), dtype=np.uint64)
    boxes = np.zeros((max(nbox, 1), 8), dtype=np.int64)
    offsets = np.zeros((5, nbox + 1), dtype=np.int64)
    tot = sum(st["list_len"].values())
    entries = np.zeros(max(tot, 1), dtype=np.int64)
    _check(lib().rpy_plan_export(plan, perm.ctypes.data, keys.ctypes.data, boxes.ctypes.data,
                                 offsets.ctypes.data, entries.ctypes.data))
    lists = {}
    e = 0
    for i, name in enumerate(LIST_NAMES):
        cnt = st["list_len"][name]
        lists[name] = (offsets[i].copy(), entries[e:e + cnt].copy())
        e += cnt
    return {"perm": perm[:n], "keys": keys[:n], "boxes": boxes[:nbox], "lists": lists}


def rpy_plan_set_timing(plan, enable):
    _check(lib().rpy_plan_set_timing(plan, int(enable)))


def rpy_plan_timings(plan):
    t = rpy_timings_t()
    _check(lib().rpy_plan_timings(plan, C.byref(t)))
    return {"ms": dict(zip(PHASES, list(t.ms))), "launches": dict(zip(PHASES, list(t.launches))),
            "passes": t.passes, "p2p_mc_ms": t.p2p_mc_ms, "p2p_mc_launches": t.p2p_mc_launches,
            "p2p_mc_rhs": t.p2p_mc_rhs}


def rpy_plan_inject_error(plan, phase):
    _check(lib().rpy_plan_inject_error(plan, int(phase)))


def rpy_plan_free(plan):
    if plan:
        lib().rpy_plan_free(plan)


# ---- torch convenience ----------------------------------------------------
class Plan:
    """A reusable RPY matvec plan over device-resident bead positions.

    positions: torch float64 CUDA tensor [n, 3] (or several systems
    concatenated, with `counts`).  The plan issues work on torch's current
    stream at construction time unless `stream` is given.
    """

    def __init__(self, positions, a, eta=1.0, eps=1e-6, precision="fp64", leaf_size=0, order=0,
                 max_depth=0, counts=None, stream=None, m2l="auto", nrhs=0, w_direct=0, eval_mode="auto", tune=0):
        import torch
        if not (isinstance(positions, torch.Tensor) and positions.is_cuda and positions.dtype == torch.float64):
            raise TypeError("positions must be a float64 CUDA tensor")
        pos = positions.contiguous()
        if pos.dim() != 2 or pos.shape[1] != 3:
            raise ValueError("positions must have shape [n, 3]")
        prec = {"fp64": PREC_FP64, "mixed": PREC_MIXED}[precision] if isinstance(precision, str) else precision
        if stream is None:
            stream = torch.cuda.current_stream(pos.device).cuda_stream
        self.device = pos.device
        self.stream = stream
        self.options = make_options(prec, leaf_size, order, max_depth, C.c_void_p(stream) if stream else None, m2l,
                                    nrhs, w_direct, eval_mode, tune)
        self.n = int(pos.shape[0])
        self.counts = [self.n] if counts is None else [int(c) for c in counts]
        if sum(self.counts) != self.n:
            raise ValueError("counts do not add up to the number of beads")
        with torch.cuda.device(self.device):
            if counts is None:
                self.handle = rpy_plan(self.n, pos.data_ptr(), a, eta, eps, self.options)
            else:
                self.handle = rpy_plan_batched(self.counts, pos.data_ptr(), a, eta, eps, self.options)
        self.a, self.eta, self.eps = float(a), float(eta), float(eps)

    def matvec(self, forces, out=None):
        """forces: float64 CUDA tensor [nrhs, n, 3] or [n, 3]; returns velocities of the same shape."""
        import torch
        if not (forces.is_cuda and forces.dtype == torch.float64):
            raise TypeError("forces must be a float64 CUDA tensor")
        F = forces.contiguous()
        squeeze = F.dim() == 2
        if squeeze:
            F = F.unsqueeze(0)
        if F.shape[1:] != (self.n, 3):
            raise ValueError(f"forces must have shape [nrhs, {self.n}, 3]")
        if out is None:
            out = torch.empty_like(F)
        with torch.cuda.device(self.device):
            rpy_matvec(self.handle, F.shape[0], F.data_ptr(), out.data_ptr())
        return out[0] if squeeze else out

    def sqrt_matvec(self, z, tol=1e-6, max_iter=50, out=None):
        """y = D^{1/2} z (Lanczos, rpy_sqrt_matvec).  z: float64 CUDA tensor
        [nrhs, n, 3] or [n, 3].  Returns (y, info)."""
        import torch
        if not (z.is_cuda and z.dtype == torch.float64):
            raise TypeError("z must be a float64 CUDA tensor")
        Z = z.contiguous()
        squeeze = Z.dim() == 2
        if squeeze:
            Z = Z.unsqueeze(0)
        if Z.shape[1:] != (self.n, 3):
            raise ValueError(f"z must have shape [nrhs, {self.n}, 3]")
        if out is None:
            out = torch.empty_like(Z)
        with torch.cuda.device(self.device):
            info = rpy_sqrt_matvec(self.handle, Z.shape[0], Z.data_ptr(), out.data_ptr(), tol, max_iter)
        return (out[0] if squeeze else out), info

    def stats(self):
        return rpy_plan_stats(self.handle)

    def export(self):
        return rpy_plan_export(self.handle)

    def set_timing(self, enable=True):
        """True/1: per-phase events with the normal concurrency; 2: phases
        run one after another on the plan stream (isolated phase times)."""
        rpy_plan_set_timing(self.handle, int(enable))

    def timings(self):
        return rpy_plan_timings(self.handle)

    def inject_error(self, phase):
        """Failure-path testing: the next matvec pass reports a HIP error at
        `phase` (a name from PHASES or its index; -1 clears), or with
        phase "alloc" the next matvec-workspace allocation fails."""
        if phase == "alloc":
            phase = RPY_INJECT_ALLOC
        elif isinstance(phase, str):
            phase = PHASES.index(phase)
        if not (-1 <= int(phase) < len(PHASES) or phase == RPY_INJECT_ALLOC):
            raise ValueError(f"phase must be -1, 'alloc' or one of {PHASES}")
        rpy_plan_inject_error(self.handle, phase)

    def free(self):
        if getattr(self, "handle", None):
            rpy_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        # at interpreter shutdown the HIP runtime may already be tearing down:
        # a plan still alive then is left to the process exit
        import sys
        if sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass
