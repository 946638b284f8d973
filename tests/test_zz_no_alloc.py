"""lam_assemble_static (the fast assembly for callers that cannot allocate)
against lam_assemble, through the C ABI.

Its kernels are lam_assemble's with the scratch regions in the library's
static device array, so its values must equal lam_assemble's bit for bit, on
consecutive calls whose plans differ (the second call smaller, so it runs on
the array's stale contents from the first), and it must write nothing into
the caller's workspace (the array really holds the scratch).  The smaller
plates are also checked against the CPU oracle (relative Frobenius <= 1e-12).
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_1905_05417_amd import workloads as W

pytestmark = pytest.mark.gpu

LAM_ESCRATCH = -8


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_05417_amd import lamasm
    lamasm.lib()
    return lamasm


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _static_call(L, plan, C, th):
    """Fresh workspace (tables uploaded, the rest a byte pattern), one
    lam_assemble_static call; returns (values, workspace before, after)."""
    ws = torch.full((plan.ws_bytes,), 0xA5, dtype=torch.uint8, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.lib().lam_plan_upload(plan._h, ws.data_ptr(), plan.ws_bytes, stream) == 0
    before = ws.clone()
    out = torch.full((plan.nnz,), float("nan"), dtype=torch.float64, device="cuda")
    st = L.lib().lam_assemble_static(plan._h, ws.data_ptr(), plan.ws_bytes, C.data_ptr(), th.data_ptr(),
                                     out.data_ptr(), plan.nnz, stream)
    assert st == 0, L.lib().lam_status_string(st)
    torch.cuda.synchronize()
    return out, before, ws


def _medium():
    rng = np.random.default_rng(901)
    lam = W.plate(2, 14, 2, list(rng.uniform(0, 180, 6)), [W.material(W.CARBON), W.material(W.GLASS)],
                  [0, 1, 1, 0, 0, 1], ne2=11, name="static_medium")
    lam.ng = (3, 3, 3)
    return lam


def _harmonic_small():
    rng = np.random.default_rng(903)
    return W.random_small(rng, max_ply=4, n_mat=2, anisotropic=False)


CALLS = [(_medium, "ply"), (W.config_q1_8x8, "bucket"), (_harmonic_small, "harmonic5")]


def test_static_equals_assemble_on_consecutive_calls(oracle, L):
    runs = []
    for make, mode in CALLS:
        lam = make()
        runs.append((lam, L.Plan(lam, set_mode=mode)))
    runs.sort(key=lambda r: -r[1].nnz)  # each call smaller than the one before
    for i, (lam, plan) in enumerate(runs):
        print("call %d: %s %s nnz %d" % (i, lam.name, plan.set_mode, plan.nnz), flush=True)
        if i > 0:
            assert plan.nnz < prev_nnz
        C, th = _dev(lam.C), _dev(lam.theta)
        ref = plan.assemble(C, th)
        torch.cuda.synchronize()
        out, before, after = _static_call(L, plan, C, th)
        assert torch.equal(out.view(torch.int64), ref.view(torch.int64))
        assert torch.equal(before, after), "lam_assemble_static wrote into the workspace"
        if plan.nnz < 200000:
            rp, ci, vals = oracle.assemble(lam)
            got = out.cpu().numpy()
            rel = float(np.linalg.norm(got - vals) / np.linalg.norm(vals))
            print("  rel vs oracle %.3e" % rel, flush=True)
            assert rel <= 1e-12
        prev_nnz = plan.nnz


def test_static_rejects_plans_beyond_its_scratch(L):
    """Degree 3 on 128x128 elements: 819,025 in-plane nonzeros of moments
    (236 MB) exceed the 128 MiB array; the call returns LAM_ESCRATCH before
    launching anything."""
    lam = W.plate(3, 128, 1, [0.0], [W.material(W.CARBON)], [0], name="too_big")
    plan = L.Plan(lam, set_mode="bucket")
    C, th = _dev(lam.C), _dev(lam.theta)
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.lib().lam_assemble_static(plan._h, plan.ws.data_ptr(), plan.ws_bytes, C.data_ptr(), th.data_ptr(),
                                     out.data_ptr(), plan.nnz, stream)
    assert st == LAM_ESCRATCH
