"""ctypes binding of the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product path never imports this module.

A laminate is passed as any object with the attributes
  p1, k1, p2, k2, q, k3   degrees and open knot vectors on [0,1]
  jac                     3x3 constant map gradient DF
  iface                   n_ply+1 ply interfaces in the thickness parameter
  ply_mat, theta          material index and angle (radians) of every ply
  C                       (n_mat, 6, 6) Voigt matrices in material axes; with
                          mat_field, (n_mat, n1*n2, 6, 6): one per in-plane function
  ng                      Gauss points (in-plane 1, in-plane 2, per z cell); 0 = degree+1
and optionally (a curved extruded shell, F = S(xi1, xi2) + xi3 a_ext)
  ctrl                    (n1*n2, 3) control points of S (in-plane function order)
  weights                 (n1*n2,) NURBS weights, or None
  a_ext                   (3,) extrusion vector
  mat_field               True: C varies in the plane as above
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("p1", ctypes.c_int32), ("p2", ctypes.c_int32), ("q", ctypes.c_int32),
        ("nk1", ctypes.c_int32), ("nk2", ctypes.c_int32), ("nk3", ctypes.c_int32),
        ("k1", _dp), ("k2", _dp), ("k3", _dp),
        ("J", ctypes.c_double * 9),
        ("n_ply", ctypes.c_int32),
        ("iface", _dp),
        ("ply_mat", _i32p),
        ("ply_theta", _dp),
        ("n_mat", ctypes.c_int32),
        ("C", _dp),
        ("ng1", ctypes.c_int32), ("ng2", ctypes.c_int32), ("ngz", ctypes.c_int32),
        ("ctrl", _dp), ("wts", _dp), ("a", ctypes.c_double * 3), ("mat_field", ctypes.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        if _LIB.startswith(_HERE) and (not os.path.exists(_LIB) or
                                       os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.or_gauss_legendre.argtypes = [ctypes.c_int, _dp, _dp]
        L.or_bspline_eval.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, _dp, _dp]
        L.or_rotate_voigt.argtypes = [_dp, ctypes.c_double, _dp]
        L.or_rotate_voigt_dtheta.argtypes = [_dp, ctypes.c_double, _dp]
        L.or_pattern_size.argtypes = [ctypes.POINTER(_Problem), _i64p]
        L.or_pattern_size.restype = ctypes.c_int64
        L.or_pattern.argtypes = [ctypes.POINTER(_Problem), _i64p, _i32p]
        L.or_assemble.argtypes = [ctypes.POINTER(_Problem), _i64p, _i32p, _dp, ctypes.c_int]
        L.or_assemble_rows.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int64, _i64p, _i64p, _i32p, _dp,
                                       ctypes.c_int]
        L.or_grad_D.argtypes = [ctypes.POINTER(_Problem), _i64p, _i32p, _dp, _dp, ctypes.c_int]
        L.or_grad_uu.argtypes = [ctypes.POINTER(_Problem), _dp, _dp, ctypes.c_int]
        L.or_grad_material.argtypes = [ctypes.c_int32, _i32p, _dp, ctypes.c_int32, _dp, _dp, _dp, _dp]
        L.or_P_pair.argtypes = [ctypes.POINTER(_Problem), _dp, ctypes.c_int, ctypes.c_int, _dp]
        L.or_Q_pair.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        L.or_surface_eval.argtypes = [ctypes.POINTER(_Problem), ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        _lib = L
    return _lib


class using_library:
    """Temporarily bind every function of this module to another build of the
    oracle (the mutation tests compile planted-mistake copies of oracle.c)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib, _LIB
        self.saved = (_lib, _LIB)
        _lib, _LIB = None, self.path
        return lib()

    def __exit__(self, *exc):
        global _lib, _LIB
        _lib, _LIB = self.saved
        return False


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


class _Bound:
    """A laminate converted to the C struct; holds the arrays it points into."""

    def __init__(self, lam):
        self.k1 = np.ascontiguousarray(lam.k1, dtype=np.float64)
        self.k2 = np.ascontiguousarray(lam.k2, dtype=np.float64)
        self.k3 = np.ascontiguousarray(lam.k3, dtype=np.float64)
        self.iface = np.ascontiguousarray(lam.iface, dtype=np.float64)
        self.ply_mat = np.ascontiguousarray(lam.ply_mat, dtype=np.int32)
        self.theta = np.ascontiguousarray(lam.theta, dtype=np.float64)
        self.C = np.ascontiguousarray(np.asarray(lam.C, dtype=np.float64).reshape(-1, 36))
        ctrl = getattr(lam, "ctrl", None)
        wts = getattr(lam, "weights", None)
        self.ctrl = None if ctrl is None else np.ascontiguousarray(np.asarray(ctrl, dtype=np.float64).reshape(-1))
        self.wts = None if wts is None else np.ascontiguousarray(np.asarray(wts, dtype=np.float64).reshape(-1))
        self.mat_field = int(bool(getattr(lam, "mat_field", False)))
        n_mat = int(np.asarray(lam.C).shape[0])
        ng = tuple(getattr(lam, "ng", (0, 0, 0)))
        J = np.asarray(lam.jac, dtype=np.float64).reshape(9)
        s = _Problem()
        s.p1, s.p2, s.q = int(lam.p1), int(lam.p2), int(lam.q)
        s.nk1, s.nk2, s.nk3 = len(self.k1), len(self.k2), len(self.k3)
        s.k1, s.k2, s.k3 = _p(self.k1), _p(self.k2), _p(self.k3)
        for a in range(9):
            s.J[a] = float(J[a])
        s.n_ply = len(self.theta)
        s.iface = _p(self.iface)
        s.ply_mat = _p(self.ply_mat, _i32p)
        s.ply_theta = _p(self.theta)
        s.n_mat = n_mat
        s.C = _p(self.C)
        s.ng1, s.ng2, s.ngz = (int(g) for g in ng)
        s.ctrl = None if self.ctrl is None else _p(self.ctrl)
        s.wts = None if self.wts is None else _p(self.wts)
        a = getattr(lam, "a_ext", None)
        for k in range(3):
            s.a[k] = 0.0 if a is None else float(a[k])
        s.mat_field = self.mat_field
        self.n_mat = n_mat
        self.s = s

    def ref(self):
        return ctypes.byref(self.s)


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle: %s rejected its input (rc=%d)" % (what, rc))


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().or_gauss_legendre(n, _p(x), _p(w)), "gauss_legendre")
    return x, w


def bspline_eval(p, knots, x):
    t = np.ascontiguousarray(knots, dtype=np.float64)
    n = len(t) - p - 1
    N = np.zeros(n)
    dN = np.zeros(n)
    _check(lib().or_bspline_eval(p, len(t), _p(t), float(x), _p(N), _p(dN)), "bspline_eval")
    return N, dN


def rotate(C6, theta):
    C = np.ascontiguousarray(C6, dtype=np.float64).reshape(36)
    D = np.zeros(36)
    lib().or_rotate_voigt(_p(C), float(theta), _p(D))
    return D.reshape(6, 6)


def rotate_dtheta(C6, theta):
    C = np.ascontiguousarray(C6, dtype=np.float64).reshape(36)
    D = np.zeros(36)
    lib().or_rotate_voigt_dtheta(_p(C), float(theta), _p(D))
    return D.reshape(6, 6)


def pattern(lam):
    b = _Bound(lam)
    nrows = ctypes.c_int64(0)
    nnz = lib().or_pattern_size(b.ref(), ctypes.byref(nrows))
    if nnz < 0:
        raise ValueError("oracle: invalid laminate")
    rowptr = np.zeros(nrows.value + 1, dtype=np.int64)
    colind = np.zeros(nnz, dtype=np.int32)
    _check(lib().or_pattern(b.ref(), _p(rowptr, _i64p), _p(colind, _i32p)), "pattern")
    return rowptr, colind


def assemble(lam, nthreads=0, pattern_=None):
    """Full standard assembly; returns (rowptr int64, colind int32, vals float64)."""
    rowptr, colind = pattern(lam) if pattern_ is None else pattern_
    b = _Bound(lam)
    vals = np.zeros(len(colind))
    _check(lib().or_assemble(b.ref(), _p(rowptr, _i64p), _p(colind, _i32p), _p(vals), int(nthreads)), "assemble")
    return rowptr, colind, vals


def assemble_rows(lam, rows, nthreads=0):
    """Selected rows; returns (ptr int64[len(rows)+1], colind int32, vals float64)."""
    b = _Bound(lam)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    L = lib()
    _check(L.or_assemble_rows(b.ref(), len(rows), _p(rows, _i64p), _p(ptr, _i64p), None, None, 0), "rows")
    col = np.zeros(int(ptr[-1]), dtype=np.int32)
    vals = np.zeros(int(ptr[-1]))
    _check(L.or_assemble_rows(b.ref(), len(rows), _p(rows, _i64p), _p(ptr, _i64p), _p(col, _i32p), _p(vals),
                              int(nthreads)), "rows")
    return ptr, col, vals


def grad_D(lam, rowptr, colind, G, nthreads=0):
    """dL/dD_l (n_ply, 6, 6) for L = sum(G * vals)."""
    b = _Bound(lam)
    G = np.ascontiguousarray(G, dtype=np.float64)
    out = np.zeros(36 * len(b.theta))
    _check(lib().or_grad_D(b.ref(), _p(rowptr, _i64p), _p(colind, _i32p), _p(G), _p(out), int(nthreads)), "grad_D")
    return out.reshape(-1, 6, 6)


def grad_D_uu(lam, u, nthreads=0):
    """dL/dD_l (n_ply, 6, 6) for L = u^T K u, without forming G or K."""
    b = _Bound(lam)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(36 * len(b.theta))
    _check(lib().or_grad_uu(b.ref(), _p(u), _p(out), int(nthreads)), "grad_uu")
    return out.reshape(-1, 6, 6)


def grad_material(lam, dLdD):
    """(dL/dC (n_mat,6,6), dL/dtheta (n_ply,)) from dL/dD_l."""
    b = _Bound(lam)
    M = np.ascontiguousarray(dLdD, dtype=np.float64).reshape(-1)
    gC = np.zeros(b.C.size)
    gT = np.zeros(len(b.theta))
    _check(lib().or_grad_material(len(b.theta), _p(b.ply_mat, _i32p), _p(b.theta), b.C.shape[0], _p(b.C), _p(M),
                                  _p(gC), _p(gT)), "grad_material")
    return gC.reshape(-1, 6, 6), gT


def grad(lam, G, nthreads=0, pattern_=None):
    rowptr, colind = pattern(lam) if pattern_ is None else pattern_
    return grad_material(lam, grad_D(lam, rowptr, colind, G, nthreads))


def surface_eval(lam, x1, x2):
    """(S, dS/dxi1, dS/dxi2) of the laminate's in-plane map at (x1, x2)."""
    b = _Bound(lam)
    x, t1, t2 = np.zeros(3), np.zeros(3), np.zeros(3)
    _check(lib().or_surface_eval(b.ref(), float(x1), float(x2), _p(x), _p(t1), _p(t2)), "surface_eval")
    return x, t1, t2


def P_pair(lam, D, i_s, j_s):
    """[alpha][beta][r][s] 2D operator for in-plane pair (i_s, j_s) and 6x6 D."""
    b = _Bound(lam)
    Dv = np.ascontiguousarray(D, dtype=np.float64).reshape(36)
    out = np.zeros(36)
    _check(lib().or_P_pair(b.ref(), _p(Dv), int(i_s), int(j_s), _p(out)), "P_pair")
    return out.reshape(2, 2, 3, 3)


def Q_pair(lam, ply, i_t, j_t):
    """[alpha][beta] 1D operator of ply `ply` for thickness pair (i_t, j_t)."""
    b = _Bound(lam)
    out = np.zeros(4)
    _check(lib().or_Q_pair(b.ref(), int(ply), int(i_t), int(j_t), _p(out)), "Q_pair")
    return out.reshape(2, 2)


def to_scipy(rowptr, colind, vals, n_rows):
    import scipy.sparse as sp
    return sp.csr_matrix((vals, colind, rowptr), shape=(n_rows, n_rows))
