"""The C-ABI library loads without a GPU and exports every function that the
public header declares (no device call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lamasm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"LAM_API\s+[\w\s\*]*?\b(lam_\w+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("lam_plan_create", "lam_pattern", "lam_assemble", "lam_assemble_standard", "lam_adjoint",
                 "lam_batch_create", "lam_batch_assemble"):
        assert must in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    from paper_1905_05417_amd import lamasm
    try:
        lib = lamasm.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip("library not built: %s" % e)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(lamasm.EXPORTED) <= set(_declared())


def test_status_strings_and_version_without_gpu():
    from paper_1905_05417_amd import lamasm
    try:
        lib = lamasm.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip("library not built: %s" % e)
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.lam_status_string(code)
    assert lib.lam_version()


def test_plan_validation_errors():
    """Descriptor checks happen on the host in lam_plan_create."""
    from paper_1905_05417_amd import lamasm, workloads as W
    try:
        lamasm.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip("library not built: %s" % e)

    def status(lam, mode="bucket"):
        d, keep = lamasm._make_desc(lam, mode)
        h = ctypes.c_void_p()
        st = lamasm.lib().lam_plan_create(ctypes.byref(d), ctypes.byref(h))
        if st == 0:
            lamasm.lib().lam_plan_destroy(h)
        return st

    assert status(W.config_q1_8x8()) == 0
    bad = W.config_q1_8x8()
    bad.k1 = bad.k1.copy()
    bad.k1[0] = 0.1  # not open on [0, 1]
    assert status(bad) == -2
    bad = W.config_q1_8x8()
    bad.iface = bad.iface.copy()
    bad.iface[2] = bad.iface[1]  # not strictly increasing
    assert status(bad) == -3
    bad = W.config_q1_8x8()
    bad.ply_mat = bad.ply_mat.copy()
    bad.ply_mat[0] = 5  # material index out of range
    assert status(bad) == -3
    bad = W.config_q1_8x8()
    bad.theta = bad.theta.copy()
    bad.theta[0] = float("nan")
    assert status(bad) == -4
    bad = W.config_q1_8x8()
    bad.p1 = 5
    assert status(bad) in (-2, -7)


def test_one_set_per_ply_mode_sizes(L=None):
    from paper_1905_05417_amd import lamasm, workloads as W
    try:
        lamasm.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip("library not built: %s" % e)
    lam = W.config_q1_8x8()
    for mode, sets in (("bucket", 2), ("ply", 4), ("harmonic5", 5), ("harmonic9", 9)):
        d, keep = lamasm._make_desc(lam, mode)
        h = ctypes.c_void_p()
        assert lamasm.lib().lam_plan_create(ctypes.byref(d), ctypes.byref(h)) == 0
        ns = ctypes.c_int32()
        assert lamasm.lib().lam_plan_info(h, None, None, None, ctypes.byref(ns), None, None) == 0
        lamasm.lib().lam_plan_destroy(h)
        assert ns.value == sets, (mode, ns.value)


def test_tuning_validation_and_cache_lookup():
    """Scatter tuning is validated on the host; the committed tuning cache
    resolves every benchmark plate and batch laminate to a tuning."""
    from paper_1905_05417_amd import autotune, lamasm, workloads as W
    try:
        lamasm.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip("library not built: %s" % e)
    lam = W.config_q1_8x8()
    d, keep = lamasm._make_desc(lam, "bucket")
    for t, ok in (({"tile_k": 32}, True), ({"set_slots": 4, "target_blocks": 100}, True), ({"tile_k": 86}, False),
                  ({"set_slots": 3}, False), ({"lds_kib": 200}, False)):
        h = ctypes.c_void_p()
        st = lamasm.lib().lam_plan_create_tuned(ctypes.byref(d), ctypes.byref(lamasm._make_tuning(t)), ctypes.byref(h))
        assert (st == 0) == ok, (t, st)
        if st == 0:
            lamasm.lib().lam_plan_destroy(h)
    cache = autotune.load_cache()
    if not cache:
        pytest.skip("no tuning cache")
    for lam in [W.config_p2_64x64_32ply(), W.config_p3_128x128_128ply()] + W.batch_laminates(16):
        t = autotune.lookup(lam, "bucket", cache)
        assert t is not None and set(t) <= {"tile_k", "set_slots", "target_blocks", "lds_kib"}


def test_product_cg_rank1_argument_errors():
    """lam_apply, lam_cg and lam_adjoint_rank1 reject bad arguments on the host,
    before any device work (a host buffer stands in for the workspace)."""
    import numpy as np
    from paper_1905_05417_amd import lamasm, workloads as W
    try:
        lib = lamasm.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip("library not built: %s" % e)

    def plan(mode):
        d, keep = lamasm._make_desc(W.config_q1_8x8(), mode)
        h = ctypes.c_void_p()
        assert lib.lam_plan_create(ctypes.byref(d), ctypes.byref(h)) == 0
        nr, nz, wb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        assert lib.lam_plan_info(h, ctypes.byref(nr), ctypes.byref(nz), ctypes.byref(wb), None, None, None) == 0
        return h, nr.value, wb.value

    h, n, wb = plan("bucket")
    raw = np.zeros(wb + 512, dtype=np.uint8)
    ws = raw.ctypes.data + (-raw.ctypes.data) % 256
    buf = np.zeros(max(n, 64), dtype=np.float64)
    p = buf.ctypes.data
    it, res = ctypes.c_int32(), ctypes.c_double()
    # r, p, q, z; the banded factor of every thickness line (ns lines of 3 nt rows, 3q + 3 band
    # columns); partial sums; scalars.  The 8x8 bilinear plate: ns = 81, nt = 5, q = 1
    assert lib.lam_cg_work_bytes(h) == 8 * (4 * n + 81 * 15 * 6 + 2 * 512 + 6)
    # wrong row count
    assert lib.lam_apply(h, ws, wb, p, p, p, None, n + 1, p, None) == -5
    assert lib.lam_adjoint_rank1(h, ws, wb, p, p, p, n - 1, p, p, None) == -5
    assert lib.lam_cg(h, ws, wb, p, p, None, p, p, n + 1, p, 1 << 30, 1e-8, 10, ctypes.byref(it), ctypes.byref(res),
                      None) == -5
    # missing pointers, short work buffer, bad tolerance or iteration count
    assert lib.lam_apply(h, ws, wb, p, p, None, None, n, p, None) == -1
    assert lib.lam_cg(h, ws, wb, p, p, None, p, p, n, p, 16, 1e-8, 10, ctypes.byref(it), ctypes.byref(res),
                      None) == -5
    assert lib.lam_cg(h, ws, wb, p, p, None, p, p, n, p, 1 << 30, -1.0, 10, ctypes.byref(it), ctypes.byref(res),
                      None) == -1
    assert lib.lam_cg(h, ws, wb, p, p, None, p, p, n, p, 1 << 30, 1e-8, -1, ctypes.byref(it), ctypes.byref(res),
                      None) == -1
    # short or misaligned workspace
    assert lib.lam_apply(h, ws, wb - 1, p, p, p, None, n, p, None) == -5
    assert lib.lam_apply(h, ws + 8, wb, p, p, p, None, n, p, None) == -1
    lib.lam_plan_destroy(h)
    # four set slots per chunk (one set per ply, four plies, a tuning): the product is unsupported
    d, keep = lamasm._make_desc(W.config_q1_8x8(), "ply")
    h = ctypes.c_void_p()
    assert lib.lam_plan_create_tuned(ctypes.byref(d), ctypes.byref(lamasm._make_tuning({"set_slots": 4})),
                                     ctypes.byref(h)) == 0
    nr, wbv = ctypes.c_int64(), ctypes.c_int64()
    assert lib.lam_plan_info(h, ctypes.byref(nr), None, ctypes.byref(wbv), None, None, None) == 0
    n, wb = nr.value, wbv.value
    raw = np.zeros(wb + 512, dtype=np.uint8)
    ws = raw.ctypes.data + (-raw.ctypes.data) % 256
    buf = np.zeros(n, dtype=np.float64)
    p = buf.ctypes.data
    assert lib.lam_apply(h, ws, wb, p, p, p, None, n, p, None) == -7
    lib.lam_plan_destroy(h)
