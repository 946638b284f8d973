"""Host side of the batched path (no GPU): planning, wave split, offsets and
argument checks of the C-ABI, called directly through ctypes."""
import ctypes

import numpy as np
import pytest

from paper_1905_05417_amd import workloads as W


@pytest.fixture(scope="module")
def L():
    from paper_1905_05417_amd import lamasm
    try:
        lamasm.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip("library not built: %s" % e)
    return lamasm


def _create(L, lams, wave_bytes, mode="bucket"):
    n = len(lams)
    descs = (L._Desc * n)()
    keep = []
    for i, lam in enumerate(lams):
        d, k = L._make_desc(lam, mode)
        descs[i] = d
        keep.append(k)
    h = ctypes.c_void_p()
    st = L.lib().lam_batch_create(n, descs, wave_bytes, ctypes.byref(h))
    return st, h, keep


def _info(L, h):
    nw, ws, mv, tn = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert L.lib().lam_batch_info(h, ctypes.byref(nw), ctypes.byref(ws), ctypes.byref(mv), ctypes.byref(tn)) == 0
    return nw.value, ws.value, mv.value, tn.value


def _lam(L, h, i):
    out = [ctypes.c_int32()] + [ctypes.c_int64() for _ in range(5)]
    st = L.lib().lam_batch_laminate(h, i, *[ctypes.byref(o) for o in out])
    return st, [o.value for o in out]


def test_waves_offsets_and_sizes(L, oracle):
    rng = np.random.default_rng(3)
    lams = [W.config_q1_8x8()] + [W.random_small(rng, max_ply=4) for _ in range(6)]
    for wave_bytes, expect_waves in ((0, 1), (1, len(lams)), (2_000_000, None)):
        st, h, keep = _create(L, lams, wave_bytes)
        assert st == 0
        nw, ws, mv, tn = _info(L, h)
        if expect_waves is not None:
            assert nw == expect_waves
        total = 0
        ends = {}
        prev_wave = 0
        for i, lam in enumerate(lams):
            st, (w, vo, nnz, nrows, co, to) = _lam(L, h, i)
            assert st == 0
            rp, ci = oracle.pattern(lam)
            assert nnz == len(ci) and nrows == len(rp) - 1
            assert vo % 32 == 0 and w >= prev_wave and 0 <= w < nw
            if w == prev_wave and i > 0:
                assert vo >= ends.get(w, 0)
            ends[w] = vo + nnz
            prev_wave = w
            assert co == 36 * sum(np.asarray(x.C).shape[0] for x in lams[:i])
            assert to == sum(x.n_ply for x in lams[:i])
            total += nnz
        assert tn == total and mv == max(ends.values()) and ws % 256 == 0
        assert _lam(L, h, len(lams))[0] == -1
        L.lib().lam_batch_destroy(h)


def test_bad_arguments(L):
    h = ctypes.c_void_p()
    assert L.lib().lam_batch_create(0, None, 0, ctypes.byref(h)) == -1
    lam = W.config_q1_8x8()
    bad = W.config_q1_8x8()
    bad.iface = bad.iface[::-1].copy()
    st, h, keep = _create(L, [lam, bad], 0)
    assert st == -3 and not h.value


def test_many_set_slots_unsupported(L):
    """Nine harmonic sets act on every thickness row: more than the two set
    slots per chunk the batched scatter holds."""
    rng = np.random.default_rng(8)
    lam = W.random_small(rng, p=2, q=2, max_ply=3, n_mat=1)
    st, h, keep = _create(L, [W.config_q1_8x8(), lam], 0, mode="harmonic9")
    assert st == -7 and not h.value
