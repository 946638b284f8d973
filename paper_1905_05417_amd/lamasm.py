"""Python binding of liblamasm.so (argument marshalling only).

Every step of the assembly runs in the library's HIP kernels; torch supplies
device memory and the current stream.  If the library is missing this module
raises: there is no CPU fallback.

    plan = Plan(laminate)                   # host plan + device workspace
    rowptr, colind = plan.pattern()         # CSR structure (int64, int32)
    vals = plan.assemble(C, theta)          # fast 2D x 1D assembly
    vals = plan.assemble_standard(C, theta) # standard 3D assembly, same CSR
    vals = assemble(plan, C, theta)         # differentiable in C and theta
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime the library shares

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblamasm.so")

LAM_SETS = {"bucket": 0, "harmonic5": 1, "harmonic9": 2, "ply": 3}

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)


class _Desc(ctypes.Structure):
    _fields_ = [
        ("p1", ctypes.c_int32), ("nk1", ctypes.c_int32), ("k1", _dp),
        ("p2", ctypes.c_int32), ("nk2", ctypes.c_int32), ("k2", _dp),
        ("q", ctypes.c_int32), ("nk3", ctypes.c_int32), ("k3", _dp),
        ("jac", ctypes.c_double * 9),
        ("n_ply", ctypes.c_int32),
        ("iface", _dp),
        ("ply_mat", _i32p),
        ("n_mat", ctypes.c_int32),
        ("ply_theta", _dp),
        ("ng1", ctypes.c_int32), ("ng2", ctypes.c_int32), ("ngz", ctypes.c_int32),
        ("set_mode", ctypes.c_int32),
    ]


class _Shell(ctypes.Structure):
    _fields_ = [("ctrl", _dp), ("weights", _dp), ("a", ctypes.c_double * 3), ("mat_field", ctypes.c_int32)]


def _make_shell(lam):
    """lam_shell for a curved laminate (None for an affine one) and the arrays it points into."""
    if getattr(lam, "ctrl", None) is None:
        return None, []
    ctrl = np.ascontiguousarray(np.asarray(lam.ctrl, dtype=np.float64).reshape(-1))
    keep = [ctrl]
    sh = _Shell()
    sh.ctrl = ctrl.ctypes.data_as(_dp)
    if getattr(lam, "weights", None) is not None:
        w = np.ascontiguousarray(np.asarray(lam.weights, dtype=np.float64).reshape(-1))
        keep.append(w)
        sh.weights = w.ctypes.data_as(_dp)
    a = np.asarray(lam.a_ext, dtype=np.float64).reshape(3)
    for k in range(3):
        sh.a[k] = float(a[k])
    sh.mat_field = 1 if getattr(lam, "mat_field", False) else 0
    return sh, keep


class _Tuning(ctypes.Structure):
    _fields_ = [("tile_k", ctypes.c_int32), ("set_slots", ctypes.c_int32), ("target_blocks", ctypes.c_int32),
                ("lds_kib", ctypes.c_int32)]


def _make_tuning(t):
    """lam_tuning from a dict (missing keys: automatic), or None."""
    if t is None:
        return None
    x = _Tuning()
    for k in ("tile_k", "set_slots", "target_blocks", "lds_kib"):
        setattr(x, k, int(t.get(k, 0) or 0))
    return x


_lib = None

EXPORTED = ("lam_plan_create", "lam_plan_create_tuned", "lam_plan_create_shell", "lam_plan_destroy", "lam_plan_info", "lam_plan_upload", "lam_check",
            "lam_pattern",
            "lam_assemble", "lam_assemble_static", "lam_assemble_standard", "lam_apply", "lam_cg", "lam_cg_work_bytes", "lam_adjoint", "lam_adjoint_rank1",
            "lam_batch_create", "lam_batch_create_tuned", "lam_batch_destroy", "lam_batch_info", "lam_batch_laminate", "lam_batch_upload",
            "lam_batch_pattern", "lam_batch_assemble", "lam_batch_check",
            "lam_profile_enable", "lam_profile_read", "lam_status_string", "lam_version")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblamasm.so is not built (run paper_1905_05417_amd/build.py); "
                               "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i64p = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)
        L.lam_plan_create.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(vp)]
        L.lam_plan_create_tuned.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(_Tuning), ctypes.POINTER(vp)]
        L.lam_batch_create_tuned.argtypes = [ctypes.c_int32, ctypes.POINTER(_Desc), ctypes.POINTER(_Tuning), i64,
                                             ctypes.POINTER(vp)]
        L.lam_plan_create_shell.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(_Shell), ctypes.POINTER(_Tuning),
                                            ctypes.POINTER(vp)]
        L.lam_plan_destroy.argtypes = [vp]
        L.lam_plan_destroy.restype = None
        L.lam_plan_info.argtypes = [vp, i64p, i64p, i64p, _i32p, _i32p, _i32p]
        L.lam_plan_upload.argtypes = [vp, vp, i64, vp]
        L.lam_check.argtypes = [vp, vp, i64, _i32p, vp]
        L.lam_pattern.argtypes = [vp, vp, i64, vp, vp, vp]
        L.lam_assemble.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp]
        L.lam_assemble_static.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp]
        L.lam_assemble_standard.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp]
        L.lam_adjoint.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp, vp, vp]
        L.lam_adjoint_rank1.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp, vp, vp]
        L.lam_apply.argtypes = [vp, vp, i64, vp, vp, vp, vp, i64, vp, vp]
        L.lam_cg_work_bytes.argtypes = [vp]
        L.lam_cg_work_bytes.restype = i64
        L.lam_cg.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, i64, vp, i64, ctypes.c_double, ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), vp]
        L.lam_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(_Desc), i64, ctypes.POINTER(vp)]
        L.lam_batch_destroy.argtypes = [vp]
        L.lam_batch_destroy.restype = None
        L.lam_batch_info.argtypes = [vp, _i32p, i64p, i64p, i64p]
        L.lam_batch_laminate.argtypes = [vp, ctypes.c_int32, _i32p, i64p, i64p, i64p, i64p, i64p]
        L.lam_batch_upload.argtypes = [vp, vp, i64, vp]
        L.lam_batch_pattern.argtypes = [vp, vp, i64, ctypes.c_int32, vp, vp, vp]
        L.lam_batch_assemble.argtypes = [vp, vp, i64, ctypes.c_int32, vp, vp, vp, i64, vp]
        L.lam_batch_check.argtypes = [vp, vp, i64, _i32p, vp]
        L.lam_profile_enable.argtypes = [ctypes.c_int32]
        L.lam_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.lam_status_string.argtypes = [ctypes.c_int32]
        L.lam_status_string.restype = ctypes.c_char_p
        L.lam_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


class LamError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s: %s (%d)" % (where, lib().lam_status_string(code).decode(), code))


def _check(code, where):
    if code != 0:
        raise LamError(code, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


CHECK_FLAGS = {1: "the plies of a bucket set were given different angles (each set is rotated by its first "
                  "ply's angle, so the values are not K(theta)); use set_mode 'ply' or a harmonic mode",
               2: "a harmonic5 plan was given a material that couples {11,22,33,12} with {13,23} (odd angular "
                  "harmonics are omitted, so the values are not K(theta)); use set_mode 'harmonic9'"}


def default_set_mode(lam) -> str:
    """One set per ply: exact for any angles passed at assembly (nothing is
    fixed at plan time), and the scatter's cost hardly grows with the number
    of sets.  Bucket sets ('bucket', one per distinct plan-time (material,
    angle) pair) serve fixed layups."""
    return "ply"


def _make_desc(lam, set_mode):
    """lam_laminate_desc for a laminate; returns it and the arrays it points into."""
    keep = [np.ascontiguousarray(lam.k1, dtype=np.float64),
            np.ascontiguousarray(lam.k2, dtype=np.float64),
            np.ascontiguousarray(lam.k3, dtype=np.float64),
            np.ascontiguousarray(lam.iface, dtype=np.float64),
            np.ascontiguousarray(lam.ply_mat, dtype=np.int32),
            np.ascontiguousarray(lam.theta, dtype=np.float64)]
    k1, k2, k3, iface, pm, th = keep
    d = _Desc()
    d.p1, d.nk1, d.k1 = int(lam.p1), len(k1), k1.ctypes.data_as(_dp)
    d.p2, d.nk2, d.k2 = int(lam.p2), len(k2), k2.ctypes.data_as(_dp)
    d.q, d.nk3, d.k3 = int(lam.q), len(k3), k3.ctypes.data_as(_dp)
    J = np.asarray(lam.jac, dtype=np.float64).reshape(9)
    for a in range(9):
        d.jac[a] = float(J[a])
    d.n_ply = len(th)
    d.iface = iface.ctypes.data_as(_dp)
    d.ply_mat = pm.ctypes.data_as(_i32p)
    d.n_mat = int(np.asarray(lam.C).shape[0])
    d.ply_theta = th.ctypes.data_as(_dp)
    d.ng1, d.ng2, d.ngz = (int(g) for g in getattr(lam, "ng", (0, 0, 0)))
    d.set_mode = LAM_SETS[set_mode]
    return d, keep


class Plan:
    """Host plan and device workspace for one laminate discretisation."""

    def __init__(self, lam, set_mode: str | None = None, device="cuda", tuning: dict | None = None):
        set_mode = set_mode or default_set_mode(lam)
        self.tuning = tuning
        self.lam = lam
        self.set_mode = set_mode
        d, self._keep = _make_desc(lam, set_mode)
        self._desc = d
        h = ctypes.c_void_p()
        t = _make_tuning(tuning)
        sh, keep_sh = _make_shell(lam)
        self._keep += keep_sh
        self.mat_field = bool(sh is not None and sh.mat_field)
        if sh is None:
            _check(lib().lam_plan_create_tuned(ctypes.byref(d), ctypes.byref(t) if t is not None else None,
                                               ctypes.byref(h)), "lam_plan_create")
        else:
            _check(lib().lam_plan_create_shell(ctypes.byref(d), ctypes.byref(sh),
                                               ctypes.byref(t) if t is not None else None, ctypes.byref(h)),
                   "lam_plan_create_shell")
        self._h = h
        nr, nz, wb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        ns, npl, nm = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lam_plan_info(h, ctypes.byref(nr), ctypes.byref(nz), ctypes.byref(wb), ctypes.byref(ns),
                                   ctypes.byref(npl), ctypes.byref(nm)), "lam_plan_info")
        self.n_rows, self.nnz, self.ws_bytes = nr.value, nz.value, wb.value
        self.n_sets, self.n_ply, self.n_mat = ns.value, npl.value, nm.value
        self.device = torch.device(device)
        self.ws = None
        if self.device.type == "cuda":
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            _check(lib().lam_plan_upload(h, self.ws.data_ptr(), self.ws_bytes, _stream()), "lam_plan_upload")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lam_plan_destroy(h)
            self._h = None

    def _ws(self):
        if self.ws is None:
            raise RuntimeError("plan has no device workspace")
        return self.ws

    def _inputs(self, C, theta):
        C = torch.as_tensor(C, dtype=torch.float64, device=self.device).contiguous()
        theta = torch.as_tensor(theta, dtype=torch.float64, device=self.device).contiguous()
        per = self.lam.n1 * self.lam.n2 if self.mat_field else 1
        if C.numel() != 36 * self.n_mat * per or theta.numel() != self.n_ply:
            raise ValueError("C must hold n_mat*36 values (times n1*n2 for a material field) and theta n_ply values")
        return C, theta

    def check(self):
        """Reads and clears the workspace's status flags (lam_check; waits for
        the stream) and raises if an assembly since the last check was given
        inputs the plan's sets cannot honour."""
        ws = self._ws()
        f = ctypes.c_int32()
        _check(lib().lam_check(self._h, ws.data_ptr(), self.ws_bytes, ctypes.byref(f), _stream()), "lam_check")
        if f.value:
            raise ValueError("lam_check: " + "; ".join(m for b, m in CHECK_FLAGS.items() if f.value & b))

    def pattern(self):
        ws = self._ws()
        rowptr = torch.empty(self.n_rows + 1, dtype=torch.int64, device=self.device)
        colind = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        _check(lib().lam_pattern(self._h, ws.data_ptr(), self.ws_bytes, rowptr.data_ptr(), colind.data_ptr(),
                                 _stream()), "lam_pattern")
        return rowptr, colind

    def assemble(self, C, theta, out=None):
        ws = self._ws()
        C, theta = self._inputs(C, theta)
        vals = torch.empty(self.nnz, dtype=torch.float64, device=self.device) if out is None else out
        _check(lib().lam_assemble(self._h, ws.data_ptr(), self.ws_bytes, C.data_ptr(), theta.data_ptr(),
                                  vals.data_ptr(), vals.numel(), _stream()), "lam_assemble")
        return vals

    def assemble_static(self, C, theta, out, ws=None):
        """lam_assemble_static: the fast assembly with its scratch in the
        library's static device array (no device allocation in the call; the
        output must be given).  ws: a workspace holding this plan's uploaded
        tables (default: the plan's own)."""
        ws = self._ws() if ws is None else ws
        C, theta = self._inputs(C, theta)
        _check(lib().lam_assemble_static(self._h, ws.data_ptr(), ws.numel() * ws.element_size(), C.data_ptr(),
                                         theta.data_ptr(), out.data_ptr(), out.numel(), _stream()),
               "lam_assemble_static")
        return out

    def assemble_standard(self, C, theta, out=None):
        """The same CSR values by the standard element-by-element 3D assembly
        (lam_assemble_standard, the comparator of Sec. 2.4)."""
        ws = self._ws()
        C, theta = self._inputs(C, theta)
        vals = torch.empty(self.nnz, dtype=torch.float64, device=self.device) if out is None else out
        _check(lib().lam_assemble_standard(self._h, ws.data_ptr(), self.ws_bytes, C.data_ptr(), theta.data_ptr(),
                                           vals.data_ptr(), vals.numel(), _stream()), "lam_assemble_standard")
        return vals

    def adjoint(self, C, theta, grad_vals):
        ws = self._ws()
        C, theta = self._inputs(C, theta)
        G = grad_vals.to(dtype=torch.float64).contiguous()
        gC = torch.empty(self.n_mat * 36, dtype=torch.float64, device=self.device)
        gT = torch.empty(self.n_ply, dtype=torch.float64, device=self.device)
        _check(lib().lam_adjoint(self._h, ws.data_ptr(), self.ws_bytes, C.data_ptr(), theta.data_ptr(),
                                 G.data_ptr(), G.numel(), gC.data_ptr(), gT.data_ptr(), _stream()), "lam_adjoint")
        return gC.view(self.n_mat, 6, 6), gT

    def apply(self, C, theta, u, out=None, fixed=None):
        """Matrix-free y = K u (lam_apply); K is never formed.  fixed: optional
        bool/uint8 tensor per row, Dirichlet rows (y = P K P u + (I - P) u)."""
        ws = self._ws()
        C, theta = self._inputs(C, theta)
        u = u.to(dtype=torch.float64).contiguous()
        fx = None if fixed is None else fixed.to(device=self.device, dtype=torch.uint8).contiguous()
        y = torch.empty(self.n_rows, dtype=torch.float64, device=self.device) if out is None else out
        _check(lib().lam_apply(self._h, ws.data_ptr(), self.ws_bytes, C.data_ptr(), theta.data_ptr(), u.data_ptr(),
                               None if fx is None else fx.data_ptr(), u.numel(), y.data_ptr(), _stream()),
               "lam_apply")
        return y

    def cg(self, C, theta, b, fixed=None, x0=None, tol=1e-10, max_iter=10000):
        """Conjugate gradients for K x = b with the Dirichlet rows `fixed`
        eliminated (lam_cg); returns (x, iterations, relative residual)."""
        ws = self._ws()
        C, theta = self._inputs(C, theta)
        b = b.to(dtype=torch.float64).contiguous()
        x = torch.zeros(self.n_rows, dtype=torch.float64, device=self.device) if x0 is None else \
            x0.to(dtype=torch.float64).clone()
        fx = None if fixed is None else fixed.to(device=self.device, dtype=torch.uint8).contiguous()
        nw = int(lib().lam_cg_work_bytes(self._h))
        work = torch.empty((nw + 7) // 8, dtype=torch.float64, device=self.device)
        iters, res = ctypes.c_int32(), ctypes.c_double()
        _check(lib().lam_cg(self._h, ws.data_ptr(), self.ws_bytes, C.data_ptr(), theta.data_ptr(),
                            None if fx is None else fx.data_ptr(), b.data_ptr(), x.data_ptr(), x.numel(),
                            work.data_ptr(), work.numel() * 8, float(tol), int(max_iter), ctypes.byref(iters),
                            ctypes.byref(res), _stream()), "lam_cg")
        return x, iters.value, res.value

    def adjoint_rank1(self, C, theta, u):
        """Gradient of L = u^T K u (lam_adjoint_rank1): G = u u^T is never formed."""
        ws = self._ws()
        C, theta = self._inputs(C, theta)
        u = u.to(dtype=torch.float64).contiguous()
        gC = torch.empty(self.n_mat * 36, dtype=torch.float64, device=self.device)
        gT = torch.empty(self.n_ply, dtype=torch.float64, device=self.device)
        _check(lib().lam_adjoint_rank1(self._h, ws.data_ptr(), self.ws_bytes, C.data_ptr(), theta.data_ptr(),
                                       u.data_ptr(), u.numel(), gC.data_ptr(), gT.data_ptr(), _stream()),
               "lam_adjoint_rank1")
        return gC.view(self.n_mat, 6, 6), gT

    def csr(self, vals, pattern=None):
        rowptr, colind = self.pattern() if pattern is None else pattern
        return torch.sparse_csr_tensor(rowptr, colind.to(torch.int64), vals, size=(self.n_rows, self.n_rows))


def profile_enable(on: bool = True):
    """Record HIP events around each entry point's dominant kernel."""
    _check(lib().lam_profile_enable(1 if on else 0), "lam_profile_enable")


PROFILE_SLOTS = ("assemble", "standard", "adjoint", "batch", "apply", "standard_fill")


def profile_read():
    """{slot: (ms_total, launches)} since the last read, slots as PROFILE_SLOTS."""
    ms = (ctypes.c_double * len(PROFILE_SLOTS))()
    n = (ctypes.c_int64 * len(PROFILE_SLOTS))()
    _check(lib().lam_profile_read(ms, n), "lam_profile_read")
    return {k: (ms[i], n[i]) for i, k in enumerate(PROFILE_SLOTS)}


class BatchPlan:
    """Many laminates assembled wave by wave (lam_batch_*).

    Laminate i's values are exactly those of Plan(lams[i]).assemble.  Waves
    are runs of consecutive laminates whose values plus scratch fit
    wave_bytes (0: everything in one wave)."""

    def __init__(self, lams, set_mode: str | None = "bucket", wave_bytes: int = 0, device="cuda", tunings=None):
        self.lams = list(lams)
        n = len(self.lams)
        descs = (_Desc * n)()
        self._keep = []
        for i, lam in enumerate(self.lams):
            d, keep = _make_desc(lam, set_mode or default_set_mode(lam))
            descs[i] = d
            self._keep.append(keep)
        h = ctypes.c_void_p()
        tarr = None
        if tunings is not None:
            tarr = (_Tuning * n)()
            for i, t in enumerate(tunings):
                tarr[i] = _make_tuning(t or {})
        _check(lib().lam_batch_create_tuned(n, descs, tarr, int(wave_bytes), ctypes.byref(h)), "lam_batch_create")
        self._h = h
        nw, wb, mv, tn = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lam_batch_info(h, ctypes.byref(nw), ctypes.byref(wb), ctypes.byref(mv), ctypes.byref(tn)),
               "lam_batch_info")
        self.n, self.n_waves, self.ws_bytes = n, nw.value, wb.value
        self.max_wave_vals, self.total_nnz = mv.value, tn.value
        self.wave, self.vals_offset, self.nnz, self.n_rows, self.c_offset, self.t_offset = ([] for _ in range(6))
        for i in range(n):
            w, vo, nz, nr, co, to = (ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(),
                                     ctypes.c_int64(), ctypes.c_int64())
            _check(lib().lam_batch_laminate(h, i, ctypes.byref(w), ctypes.byref(vo), ctypes.byref(nz),
                                            ctypes.byref(nr), ctypes.byref(co), ctypes.byref(to)),
                   "lam_batch_laminate")
            for lst, v in ((self.wave, w), (self.vals_offset, vo), (self.nnz, nz), (self.n_rows, nr),
                           (self.c_offset, co), (self.t_offset, to)):
                lst.append(v.value)
        self.wave_vals = [0] * self.n_waves
        for i in range(n):
            self.wave_vals[self.wave[i]] = max(self.wave_vals[self.wave[i]], self.vals_offset[i] + self.nnz[i])
        self.device = torch.device(device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        _check(lib().lam_batch_upload(h, self.ws.data_ptr(), self.ws_bytes, _stream()), "lam_batch_upload")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lam_batch_destroy(h)
            self._h = None

    def pack(self, Cs=None, thetas=None):
        """Device C_all and theta_all from per-laminate tensors (default: the laminates' own)."""
        Cs = [lam.C for lam in self.lams] if Cs is None else Cs
        thetas = [lam.theta for lam in self.lams] if thetas is None else thetas
        C_all = torch.cat([torch.as_tensor(np.asarray(c, dtype=np.float64)).reshape(-1) for c in Cs])
        th_all = torch.cat([torch.as_tensor(np.asarray(t, dtype=np.float64)).reshape(-1) for t in thetas])
        return C_all.to(self.device), th_all.to(self.device)

    def pattern(self, i):
        rowptr = torch.empty(self.n_rows[i] + 1, dtype=torch.int64, device=self.device)
        colind = torch.empty(self.nnz[i], dtype=torch.int32, device=self.device)
        _check(lib().lam_batch_pattern(self._h, self.ws.data_ptr(), self.ws_bytes, i, rowptr.data_ptr(),
                                       colind.data_ptr(), _stream()), "lam_batch_pattern")
        return rowptr, colind

    def assemble_wave(self, wave, C_all, th_all, out):
        """Enqueue wave `wave` into out (device float64, >= wave_vals[wave])."""
        _check(lib().lam_batch_assemble(self._h, self.ws.data_ptr(), self.ws_bytes, int(wave), C_all.data_ptr(),
                                        th_all.data_ptr(), out.data_ptr(), out.numel(), _stream()),
               "lam_batch_assemble")
        return out

    def check(self):
        """Reads and clears every laminate's status flags (lam_batch_check;
        waits for the stream) and raises if an assembly since the last check
        was given angles that a laminate's bucket sets cannot honour."""
        f = ctypes.c_int32()
        _check(lib().lam_batch_check(self._h, self.ws.data_ptr(), self.ws_bytes, ctypes.byref(f), _stream()),
               "lam_batch_check")
        if f.value:
            raise ValueError("lam_batch_check: " + "; ".join(m for b, m in CHECK_FLAGS.items() if f.value & b))

    def laminate_vals(self, i, wave_buf):
        o = self.vals_offset[i]
        return wave_buf[o:o + self.nnz[i]]

    def assemble(self, C_all=None, th_all=None):
        """All laminates, wave by wave; returns a list of per-laminate value tensors (copies)."""
        if C_all is None:
            C_all, th_all = self.pack()
        out = [None] * self.n
        buf = torch.empty(self.max_wave_vals, dtype=torch.float64, device=self.device)
        for w in range(self.n_waves):
            self.assemble_wave(w, C_all, th_all, buf)
            self.check()
            for i in range(self.n):
                if self.wave[i] == w:
                    out[i] = self.laminate_vals(i, buf).clone()
        return out


class _Assemble(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C, theta, plan):
        if plan.set_mode == "bucket":
            raise ValueError("assemble(): a bucket plan groups plies by their plan-time angles, so it cannot follow "
                             "per-ply angle changes; differentiate through a 'ply' or harmonic plan")
        ctx.plan = plan
        ctx.save_for_backward(C, theta)
        vals = plan.assemble(C.detach(), theta.detach())
        if plan.set_mode == "harmonic5":
            plan.check()  # the five-term split needs materials without {11,22,33,12}-{13,23} coupling
        return vals

    @staticmethod
    def backward(ctx, grad_vals):
        C, theta = ctx.saved_tensors
        gC, gT = ctx.plan.adjoint(C.detach(), theta.detach(), grad_vals)
        return gC.view_as(C), gT.view_as(theta), None


def assemble(plan: Plan, C: torch.Tensor, theta: torch.Tensor) -> torch.Tensor:
    """CSR values of K(C, theta); differentiable in C (n_mat,6,6) and theta (n_ply,).

    The backward is lam_adjoint.  Bucket plans are refused (their sets fix the
    ply angles' grouping at plan time); harmonic5 plans are checked on the
    device for materials the five-term split cannot represent."""
    return _Assemble.apply(C, theta, plan)
