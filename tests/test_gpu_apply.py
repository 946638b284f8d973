"""Matrix-free y = K u (lam_apply) against the CPU oracle's assembled K.

Bar: relative Frobenius error <= 1e-12 on every case (the product is a
reordering of the same sums).  Small laminates: the whole y against the
oracle's K times u.  The 64x64 32-ply plate: sampled rows of the oracle's K
times u, and the GPU's own assembled K times u on the GPU.  Invariants: a
rigid translation has K u = 0; K is symmetric, so v^T (K u) = u^T (K v).
"""
import numpy as np
import pytest
import torch

from paper_1905_05417_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_05417_amd import lamasm
    lamasm.lib()
    return lamasm


def _mats(lam):
    return (torch.tensor(np.asarray(lam.C, dtype=np.float64), device="cuda"),
            torch.tensor(np.asarray(lam.theta, dtype=np.float64), device="cuda"))


@pytest.mark.parametrize("case", range(8))
def test_apply_matches_oracle(oracle, L, case):
    rng = np.random.default_rng(7100 + case)
    lam = W.config_q1_8x8() if case == 0 else W.random_small(rng, max_ply=6, n_mat=2)
    # five harmonics are exact for orthotropic materials only (the q1 plate's carbon)
    mode = "harmonic5" if case == 0 else ("bucket", "ply", "harmonic9", "ply")[case % 4]
    tuning = ({}, {"target_blocks": 1}, {"target_blocks": 3, "tile_k": 20}, {})[(case // 2) % 4]
    print("case", case, mode, tuning, lam.p1, lam.p2, lam.q, lam.n_ply, flush=True)
    rp, ci, ref = oracle.assemble(lam)
    K = oracle.to_scipy(rp, ci, ref, len(rp) - 1)
    plan = L.Plan(lam, set_mode=mode, tuning=tuning)
    C, th = _mats(lam)
    u = rng.standard_normal(plan.n_rows)
    y = plan.apply(C, th, torch.tensor(u, device="cuda")).cpu().numpy()
    yr = K @ u
    rel = float(np.linalg.norm(y - yr) / np.linalg.norm(yr))
    print("  rel %.3e" % rel, flush=True)
    assert rel <= TOL


def test_apply_unsupported_plans(L):
    """Four set slots per chunk (one set per ply, four plies, a tuning): LAM_EUNSUP."""
    lam = W.config_q1_8x8()
    plan = L.Plan(lam, set_mode="ply", tuning={"set_slots": 4})
    C, th = _mats(lam)
    with pytest.raises(L.LamError):
        plan.apply(C, th, torch.zeros(plan.n_rows, dtype=torch.float64, device="cuda"))


def test_apply_translation_and_symmetry(L):
    rng = np.random.default_rng(7300)
    lam = W.random_small(rng, max_ply=6, n_mat=2)
    plan = L.Plan(lam, set_mode="bucket")
    C, th = _mats(lam)
    t = torch.zeros(plan.n_rows, dtype=torch.float64, device="cuda")
    t[0::3], t[1::3], t[2::3] = 1.0, -0.5, 0.25
    u = torch.tensor(rng.standard_normal(plan.n_rows), device="cuda")
    v = torch.tensor(rng.standard_normal(plan.n_rows), device="cuda")
    Ku, Kv, Kt = plan.apply(C, th, u), plan.apply(C, th, v), plan.apply(C, th, t)
    scale = float(Ku.norm() / u.norm())
    assert float(Kt.norm() / t.norm()) <= 1e-12 * scale
    a, b = float(v @ Ku), float(u @ Kv)
    assert abs(a - b) <= 1e-12 * float(v.norm() * Ku.norm())


def test_apply_full_plate(oracle, L):
    """64x64 32-ply degree-2 plate: 300 sampled rows of the oracle's K times u,
    and the whole y against the GPU's assembled K times u."""
    lam = W.config_p2_64x64_32ply()
    plan = L.Plan(lam, set_mode="bucket")
    C, th = _mats(lam)
    rng = np.random.default_rng(7400)
    u_np = rng.standard_normal(plan.n_rows)
    u = torch.tensor(u_np, device="cuda")
    y = plan.apply(C, th, u)
    rows = np.unique(rng.choice(plan.n_rows, size=300, replace=False))
    ptr, col, vals = oracle.assemble_rows(lam, rows)
    yr = np.add.reduceat(vals * u_np[col], ptr[:-1])
    yg = y.cpu().numpy()[rows]
    rel = float(np.linalg.norm(yg - yr) / np.linalg.norm(yr))
    print("sampled rows rel %.3e" % rel, flush=True)
    assert rel <= TOL
    rowptr, colind = plan.pattern()
    vals_g = plan.assemble(C, th)
    K = torch.sparse_csr_tensor(rowptr, colind.to(torch.int64), vals_g, size=(plan.n_rows, plan.n_rows))
    y2 = torch.mv(K, u)
    rel2 = float((y - y2).norm() / y2.norm())
    print("vs assembled K on the GPU rel %.3e" % rel2, flush=True)
    assert rel2 <= TOL


def _clamped_rows(lam, n_rows):
    """Rows of the functions on the first in-plane edge (i1 = 0): all
    thickness functions and components there are fixed."""
    n1 = len(lam.k1) - lam.p1 - 1
    n2 = len(lam.k2) - lam.p2 - 1
    rows = np.arange(n_rows)
    return (((rows // 3) % (n1 * n2)) % n1 == 0)


@pytest.mark.parametrize("case", range(4))
def test_apply_dirichlet_and_cg(oracle, L, case):
    """Eliminated operator P K P u + (I - P) u against the oracle's K, and CG
    for the clamped laminate to a recurrence residual of 1e-12: the normwise
    backward error of x against the oracle's K_ff, ||K_ff x_f - b_f|| /
    (||K_ff|| ||x_f|| + ||b_f||) with the Frobenius norm, is below 1e-12 (the
    true residual itself can exceed the recurrence's by cond(K_ff) times the
    rounding of the products), and the fixed entries of x are zero."""
    rng = np.random.default_rng(7500 + case)
    lam = W.config_q1_8x8() if case == 0 else W.random_small(rng, max_ply=5, n_mat=2)
    mode = ("bucket", "ply")[case % 2]
    rp, ci, ref = oracle.assemble(lam)
    n = len(rp) - 1
    K = oracle.to_scipy(rp, ci, ref, n)
    fixed = _clamped_rows(lam, n)
    free = ~fixed
    plan = L.Plan(lam, set_mode=mode)
    C, th = _mats(lam)
    fx = torch.tensor(fixed, device="cuda")
    u = rng.standard_normal(n)
    y = plan.apply(C, th, torch.tensor(u, device="cuda"), fixed=fx).cpu().numpy()
    yr = np.where(free, K @ np.where(free, u, 0.0), u)
    e_apply = float(np.linalg.norm(y - yr) / np.linalg.norm(yr))
    b = rng.standard_normal(n)
    x, iters, res = plan.cg(C, th, torch.tensor(b, device="cuda"), fixed=fx, tol=1e-12, max_iter=50 * n)
    x = x.cpu().numpy()
    Kff = K[free][:, free]
    r = Kff @ x[free] - b[free]
    e_cg = float(np.linalg.norm(r) / (np.sqrt(Kff.multiply(Kff).sum()) * np.linalg.norm(x[free]) +
                                      np.linalg.norm(b[free])))
    print("case %d n %d: apply rel %.2e, cg %d iterations, residual %.2e (oracle K: backward error %.2e, "
          "relative residual %.2e)" % (case, n, e_apply, iters, res, e_cg,
                                        np.linalg.norm(r) / np.linalg.norm(b[free])), flush=True)
    assert e_apply <= TOL
    assert res <= 1e-12 and e_cg <= 1e-12
    assert np.abs(x[fixed]).max() == 0.0
