"""GPU parity of the fast 2D x 1D assembly against the CPU oracle, through the C ABI.

Bar: CSR pattern bit-exact (int64 rowptr, int32 colind); values within
relative Frobenius error 1e-12 and max-abs error 1e-12 * max|K| (FP64 sums
of different order; the split itself introduces no approximation, Sec. 3).
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
    C = torch.tensor(np.asarray(lam.C, dtype=np.float64), device="cuda")
    th = torch.tensor(np.asarray(lam.theta, dtype=np.float64), device="cuda")
    return C, th


def _compare_full(oracle, L, lam, mode, tol=TOL):
    print("case", lam.name, mode, lam.p1, lam.p2, lam.q, lam.n_ply, flush=True)
    rp, ci, v = oracle.assemble(lam)
    plan = L.Plan(lam, set_mode=mode)
    grp, gci = plan.pattern()
    C, th = _mats(lam)
    gv = plan.assemble(C, th)
    torch.cuda.synchronize()
    assert np.array_equal(grp.cpu().numpy(), rp)
    assert np.array_equal(gci.cpu().numpy(), ci)
    g = gv.cpu().numpy()
    relF = np.linalg.norm(g - v) / np.linalg.norm(v)
    relM = np.abs(g - v).max() / np.abs(v).max()
    print("  nnz", len(v), "sets", plan.n_sets, "relF %.3e relmax %.3e" % (relF, relM), flush=True)
    assert relF <= tol and relM <= tol
    return plan, g


def test_q1_8x8_4ply(oracle, L):
    lam = W.config_q1_8x8()
    for mode in ("bucket", "harmonic5", "harmonic9"):
        _compare_full(oracle, L, lam, mode)


@pytest.mark.parametrize("seed", range(6))
def test_random_small_anisotropic(oracle, L, seed):
    """Nonuniform knots with a repeated knot, sheared map, fully anisotropic
    materials, random angles; odd seeds put every ply in one thickness element."""
    rng = np.random.default_rng(1000 + seed)
    lam = W.random_small(rng, paper_regime=(seed % 2 == 1), max_ply=5)
    _compare_full(oracle, L, lam, "bucket")
    _compare_full(oracle, L, lam, "harmonic9")


@pytest.mark.parametrize("seed", range(3))
def test_one_set_per_ply(oracle, L, seed):
    """Every ply its own set, the angles read only at assembly: exact for any
    angles, including ones that differ from the plan-time values."""
    rng = np.random.default_rng(1100 + seed)
    lam = W.random_small(rng, max_ply=6, n_mat=2)
    _compare_full(oracle, L, lam, "ply")
    lam.theta = rng.uniform(0, np.pi, size=lam.n_ply)
    _compare_full(oracle, L, lam, "ply")


def test_harmonic5_orthotropic(oracle, L):
    rng = np.random.default_rng(77)
    lam = W.random_small(rng, anisotropic=False, max_ply=5)
    _compare_full(oracle, L, lam, "harmonic5")


def test_several_tiles_ragged(oracle, L):
    """p=2 in-plane 11x7 elements, 7 plies: many Kronecker tiles, ragged last tile,
    boundary rows of every length."""
    lam = W.plate(2, 11, 2, [0, 45, -45, 90, 30, 0, 90], [W.material(W.CARBON), W.material(W.GLASS)],
                  [0, 1, 0, 1, 1, 0, 0], ne2=7, name="p2_11x7_7ply")
    _compare_full(oracle, L, lam, "bucket")
    _compare_full(oracle, L, lam, "harmonic5")


def test_p3_mixed_degrees(oracle, L):
    lam = W.plate(3, 6, 2, [0, 90, 45], [W.material(W.CARBON)], [0, 0, 0], ne2=5, p2=1, name="p3xp1")
    _compare_full(oracle, L, lam, "bucket")


def test_single_ply_single_element(oracle, L):
    """Degenerate: one in-plane element, one ply, p = q = 1."""
    lam = W.plate(1, 1, 1, [30.0], [W.material(W.CARBON)], [0], H=0.05, name="one_element")
    _compare_full(oracle, L, lam, "bucket")
    _compare_full(oracle, L, lam, "harmonic9")


def test_deterministic(oracle, L):
    lam = W.plate(2, 9, 2, [0, 90] * 3, [W.material(W.CARBON)], [0] * 6, name="det")
    plan = L.Plan(lam, set_mode="bucket")
    C, th = _mats(lam)
    a = plan.assemble(C, th).clone()
    b = plan.assemble(C, th)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def _sampled_rows(oracle, L, lam, mode, n_rand=1500, seed=5, tuning=None):
    plan = L.Plan(lam, set_mode=mode, tuning=tuning)
    print("case", lam.name, mode, tuning, "nnz", plan.nnz, flush=True)
    rowptr, colind = plan.pattern()
    C, th = _mats(lam)
    vals = plan.assemble(C, th)
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    n = plan.n_rows
    ns = lam.n1 * lam.n2
    # random rows plus structured ones: first/last rows, every component of a
    # corner, an edge and an interior in-plane function on an interface row
    special = [0, 1, 2, n - 1, n - 2, n - 3]
    for it in (0, lam.q, lam.q + 1, lam.nt // 2, lam.nt - 1):
        for is_ in (0, lam.n1 - 1, lam.n1 // 2 + lam.n1 * (lam.n2 // 2), ns - 1):
            for r in range(3):
                special.append(3 * (it * ns + is_) + r)
    rows = np.unique(np.concatenate([rng.choice(n, size=n_rand, replace=False), np.array(special)]))
    ptr, col, ref = oracle.assemble_rows(lam, rows)
    rp = rowptr.cpu().numpy()
    assert rp[-1] == plan.nnz and np.all(np.diff(rp) > 0)
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    it = torch.tensor(idx, device="cuda")
    gcol = colind[it].cpu().numpy()
    gval = vals[it].cpu().numpy()
    assert np.array_equal(gcol, col)
    relF = np.linalg.norm(gval - ref) / np.linalg.norm(ref)
    relM = np.abs(gval - ref).max() / np.abs(ref).max()
    print("  rows", len(rows), "entries", len(ref), "relF %.3e relmax %.3e" % (relF, relM), flush=True)
    assert relF <= TOL and relM <= TOL


def test_full_size_p2_64x64_32ply_sampled(oracle, L):
    _sampled_rows(oracle, L, W.config_p2_64x64_32ply(), "bucket")


def test_full_size_adjoint_plate_sampled(oracle, L):
    _sampled_rows(oracle, L, W.config_adjoint_p2_96x96_64ply(), "harmonic5", n_rand=800)


def test_full_size_adjoint_plate_sampled_one_set_per_ply(oracle, L):
    """64 plies with seeded random angles, one set per ply: every chunk holds
    one ply, groups of chunks share the block (the grouped scatter at full size)."""
    from paper_1905_05417_amd import autotune
    lam = W.config_adjoint_p2_96x96_64ply()
    _sampled_rows(oracle, L, lam, "ply", n_rand=800, tuning=autotune.lookup(lam, "bucket"))


def test_full_size_p3_128x128_128ply_sampled(oracle, L):
    """The 128-ply degree-3 plate (7.6e9 nonzeros, 60 GB of values) with the
    tuned scatter of the benchmark: sampled rows against the oracle."""
    from paper_1905_05417_amd import autotune
    lam = W.config_p3_128x128_128ply()
    _sampled_rows(oracle, L, lam, "bucket", n_rand=400, tuning=autotune.lookup(lam, "bucket"))
