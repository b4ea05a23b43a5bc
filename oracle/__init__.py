"""FP64 CPU oracle for the RPY mobility matvec -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library
(``paper_1711_02976_amd``) never imports it and shares no code with it.

Thin ctypes wrapper over ``rpy_oracle.c`` (see that file's header for the
passages of arXiv:1711.02976 each function follows and the readings taken).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpy_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

GCC_CMD = ["gcc", "-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-o", _LIB, _SRC, "-lm"]


def build(force: bool = True) -> str:
    """Compile the oracle shared library in-tree and return its path."""
    if force or not os.path.exists(_LIB):
        subprocess.run(GCC_CMD, check=True)
    return _LIB


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        # RPY_ORACLE_LIB: another build of rpy_oracle.c (the sanitizer test's)
        path = os.environ.get("RPY_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        L = C.CDLL(path)
        L.orc_rpy_block.argtypes = [_dp, C.c_double, C.c_double, _dp]
        L.orc_rpy_direct.argtypes = [C.c_int64, _dp, C.c_int, _dp, C.c_double, C.c_double,
                                     C.c_int64, C.c_void_p, _dp, C.c_int]
        L.orc_far_four_laplace.argtypes = [C.c_int64, _dp, _dp, C.c_double, C.c_double,
                                           C.c_void_p, _dp, C.c_int]
        L.orc_legendre.argtypes = [C.c_int, C.c_double, _dp]
        L.orc_ynm.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp]
        L.orc_tree_build.argtypes = [C.c_int64, _dp, C.c_int, C.c_int, C.c_double]
        L.orc_tree_build.restype = C.c_void_p
        L.orc_tree_free.argtypes = [C.c_void_p]
        L.orc_tree_sizes.argtypes = [C.c_void_p, _ip, _dp]
        L.orc_tree_export.argtypes = [C.c_void_p, _up, _ip, _ip, _ip, _ip]
        L.orc_p2m.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _dp]
        L.orc_p2l.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _dp]
        L.orc_translate.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.orc_eval_expansion.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_fmm.argtypes = [C.c_int64, _dp, C.c_int, _dp, C.c_double, C.c_double, C.c_int,
                              C.c_int, C.c_int, C.c_int64, C.c_int, _dp, C.c_int]
        L.orc_solid_monomials.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp]
        L.orc_fmm.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        L.orc_rpy_dense.argtypes = [C.c_int64, _dp, C.c_double, C.c_double, _dp]
        _lib = L
    return _lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def max_threads() -> int:
    return lib().orc_max_threads()


def rpy_block(d, a, eta):
    """3x3 RPY mobility block for separation d (Sec. 1, RPY equations)."""
    out = np.zeros(9)
    lib().orc_rpy_block(_f64(d), a, eta, out)
    return out.reshape(3, 3)


def rpy_direct(pos, forces, a, eta, targets=None, nthreads=0):
    """O(N^2) direct RPY matvec.  pos [n,3]; forces [nrhs,n,3] or [n,3].
    Returns [nrhs, nt, 3] (or [nt, 3] for a 2-D force array)."""
    pos = _f64(pos)
    F = _f64(forces)
    squeeze = F.ndim == 2
    if squeeze:
        F = F[None]
    n = pos.shape[0]
    nrhs = F.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = tg.shape[0], tg.ctypes.data
    out = np.zeros((nrhs, nt, 3))
    lib().orc_rpy_direct(n, pos, nrhs, F, a, eta, nt, tp, out, nthreads)
    return out[0] if squeeze else out


def rpy_dense(pos, a, eta):
    """Dense 3n x 3n RPY mobility matrix D (Sec. 1, RPY block equations)."""
    pos = _f64(pos)
    n = pos.shape[0]
    out = np.zeros((3 * n, 3 * n))
    lib().orc_rpy_dense(n, pos, a, eta, out)
    return out


def rpy_sqrt(pos, z, a, eta):
    """Brownian displacement directions y = D^{1/2} z (Sec. 1: the random
    displacements of the Ermak-McCammon step have covariance 2 D dt), with
    D^{1/2} = Q diag(sqrt(lambda)) Q^T from numpy's symmetric eigensolver on
    the dense D.  z [nrhs, n, 3] or [n, 3]; returns the same shape.  Raises
    if D is not positive definite (the RPY tensor is, for any positions)."""
    Z = _f64(z)
    squeeze = Z.ndim == 2
    if squeeze:
        Z = Z[None]
    n = Z.shape[1]
    lam, Q = np.linalg.eigh(rpy_dense(pos, a, eta))
    if lam.min() <= 0.0:
        raise ValueError(f"mobility matrix not positive definite (smallest eigenvalue {lam.min():.3e})")
    Y = (Q * np.sqrt(lam)) @ (Q.T @ Z.reshape(Z.shape[0], 3 * n).T)
    Y = Y.T.reshape(Z.shape)
    return Y[0] if squeeze else Y


def far_four_laplace(pos, forces, a, eta, centers=None, nthreads=0):
    """Far-field (r >= 2a) RPY via eq. (2.8) by brute force; forces [n,3]."""
    pos = _f64(pos)
    F = _f64(forces)
    out = np.zeros((pos.shape[0], 3))
    cp = None
    if centers is not None:
        cen = _f64(centers)
        cp = cen.ctypes.data
    lib().orc_far_four_laplace(pos.shape[0], pos, F, a, eta, cp, out, nthreads)
    return out


def legendre(P, x):
    out = np.zeros((P + 1) * (P + 2) // 2)
    lib().orc_legendre(P, float(x), out)
    return out


def ynm(P, theta, phi):
    re = np.zeros((P + 1) * (P + 2) // 2)
    im = np.zeros_like(re)
    lib().orc_ynm(P, float(theta), float(phi), re, im)
    return re + 1j * im


def _cplx_out(p):
    return np.zeros(2 * (p + 1) * (p + 2) // 2)


def p2m(p, src, q, c):
    out = _cplx_out(p)
    src = _f64(src)
    lib().orc_p2m(p, src.shape[0], src, _f64(q), _f64(c), out)
    return out[0::2] + 1j * out[1::2]


def p2l(p, src, q, c):
    out = _cplx_out(p)
    src = _f64(src)
    lib().orc_p2l(p, src.shape[0], src, _f64(q), _f64(c), out)
    return out[0::2] + 1j * out[1::2]


def translate(p, op, coeffs, c0, c1):
    """op: 'm2m', 'm2l' or 'l2l'; coeffs complex [(p+1)(p+2)/2]."""
    code = {"m2m": 0, "m2l": 1, "l2l": 2}[op]
    cin = np.empty(2 * coeffs.size)
    cin[0::2] = coeffs.real
    cin[1::2] = coeffs.imag
    out = _cplx_out(p)
    lib().orc_translate(p, code, cin, _f64(c0), _f64(c1), out)
    return out[0::2] + 1j * out[1::2]


def eval_expansion(p, kind, coeffs, v):
    """kind 'M' (Theorem 1) or 'L' (Theorem 2) at offset v from the centre.
    Returns (value, gradient[3], hessian[3,3])."""
    cin = np.empty(2 * coeffs.size)
    cin[0::2] = coeffs.real
    cin[1::2] = coeffs.imag
    out = np.zeros(13)
    lib().orc_eval_expansion(p, 0 if kind == "M" else 1, cin, _f64(v), out)
    return out[0], out[1:4], out[4:].reshape(3, 3)


LIST_NAMES = ("U", "V", "W", "X", "O")


class Tree:
    """Adaptive octree and interaction lists built from their definitions."""

    def __init__(self, pos, leaf_size, max_depth, a):
        pos = _f64(pos)
        L = lib()
        h = L.orc_tree_build(pos.shape[0], pos, int(leaf_size), int(max_depth), float(a))
        try:
            sizes = np.zeros(6, dtype=np.int64)
            geom = np.zeros(4)
            L.orc_tree_sizes(h, sizes, geom)
            nbox = int(sizes[0])
            n = pos.shape[0]
            self.keys = np.zeros(n, dtype=np.uint64)
            self.perm = np.zeros(n, dtype=np.int64)
            boxes = np.zeros((max(nbox, 1), 8), dtype=np.int64)
            offsets = np.zeros((5, nbox + 1), dtype=np.int64)
            entries = np.zeros(max(int(sizes[1:].sum()), 1), dtype=np.int64)
            if n > 0:
                L.orc_tree_export(h, self.keys, self.perm, boxes, offsets, entries)
        finally:
            L.orc_tree_free(h)
        self.lo = geom[:3].copy()
        self.side = float(geom[3])
        self.nbox = nbox
        self.boxes = boxes[:nbox]
        self.level = self.boxes[:, 0]
        self.anchor = self.boxes[:, 1:4]
        self.begin = self.boxes[:, 4]
        self.end = self.boxes[:, 5]
        self.parent = self.boxes[:, 6]
        self.child_begin = self.boxes[:, 7]
        self.lists = {}
        e = 0
        for i, name in enumerate(LIST_NAMES):
            cnt = int(sizes[1 + i])
            self.lists[name] = (offsets[i].copy(), entries[e:e + cnt].copy())
            e += cnt

    def is_leaf(self):
        return self.child_begin < 0

    def centers(self):
        h = self.side / (2.0 ** self.level)
        return self.lo[None, :] + (self.anchor + 0.5) * h[:, None]


def fmm(pos, forces, a, eta, p, leaf_size, w_direct, max_depth=14, nthreads=0, eval_mode=0):
    """The four-Laplace adaptive FMM (O4) in FP64.  forces [nrhs,n,3] or
    [n,3]; returns the same shape.  W-list boxes with at most w_direct beads
    are summed directly with the far formula, the others through their
    multipoles (w_direct < 0: all through multipoles); the caller chooses.
    eval_mode: 0 = Sec. 2's first evaluation approach (Theorem 2 derivatives
    per Laplace expansion, then eq. (2.8)); 1 = its second approach (one
    pre-assembled polynomial per velocity component and leaf)."""
    pos = _f64(pos)
    F = _f64(forces)
    squeeze = F.ndim == 2
    if squeeze:
        F = F[None]
    out = np.zeros_like(F)
    rc = lib().orc_fmm(pos.shape[0], pos, F.shape[0], F, a, eta, int(p), int(leaf_size),
                       int(max_depth), int(w_direct), int(eval_mode), out, nthreads)
    if rc != 0:
        raise ValueError("orc_fmm rejected its arguments")
    return out[0] if squeeze else out


def solid_monomials(P, n, m):
    """Monomial coefficients [a, b, c] (a + b + c <= P) of r^n P_n^m(cos t)
    e^{i m phi}, Condon-Shortley phase, as a complex (P+1)^3 array."""
    re = np.zeros((P + 1) ** 3)
    im = np.zeros((P + 1) ** 3)
    lib().orc_solid_monomials(int(P), int(n), int(m), re, im)
    return (re + 1j * im).reshape(P + 1, P + 1, P + 1)


def rel_l2(u, ref):
    """sqrt(sum |u_i - ref_i|^2 / sum |ref_i|^2) over targets (3-vector norm);
    the reading taken for the paper's accuracy formula (Sec. 4.3, Table 1)."""
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.sum((u - ref) ** 2) / np.sum(ref ** 2)))
