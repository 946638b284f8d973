"""Every kernel branch the C ABI accepts, against the CPU oracle.

The ABI takes thickness degrees up to 4 and any thickness knots, including
knots inside a ply (Sec. 2.4, remark on the through-thickness discretization:
the split holds for any thickness space).  These cases reach code the
benchmark plates do not:
  * layerwise q = 3 and q = 4: thickness rows of width 7 and 9, the scatter's
    generic row body, the adjoint's streaming kernel for rows of 7 and 9, the
    matrix-free product at those widths;
  * a ply holding two thickness elements (an interior knot of any
    multiplicity);
  * the LDS-mode scatter with P read from memory (more than eight sets on a
    thickness row and an LDS budget too small to stage P).
Whole-matrix parity of the 32-ply and 64-ply plates against the oracle's full
assembly closes the file.

Bar: patterns bit-exact; values within relative Frobenius and max-abs error
1e-12 (max-abs relative to max |K|); products within 1e-12; gradients within
1e-10 of the oracle's.
"""
import numpy as np
import pytest
import torch

from paper_1905_05417_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
GTOL = 1e-10


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


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _fast_full(oracle, L, lam, mode, tuning=None, ref=None):
    rp, ci, v = oracle.assemble(lam) if ref is None else ref
    plan = L.Plan(lam, set_mode=mode, tuning=tuning)
    grp, gci = plan.pattern()
    C, th = _mats(lam)
    g = plan.assemble(C, th).cpu().numpy()
    assert np.array_equal(grp.cpu().numpy(), rp) and np.array_equal(gci.cpu().numpy(), ci)
    relF = float(np.linalg.norm(g - v) / np.linalg.norm(v))
    relM = _rel(g, v)
    print("  fast %s %s: nnz %d relF %.3e relmax %.3e" % (mode, tuning, len(v), relF, relM), flush=True)
    assert relF <= TOL and relM <= TOL
    plan.check()
    return plan


def _apply_and_adjoint(oracle, L, lam, plan, ref, rng):
    rp, ci, v = ref
    C, th = _mats(lam)
    K = oracle.to_scipy(rp, ci, v, len(rp) - 1)
    u = rng.standard_normal(plan.n_rows)
    y = plan.apply(C, th, torch.tensor(u, device="cuda")).cpu().numpy()
    ry = float(np.linalg.norm(y - K @ u) / np.linalg.norm(K @ u))
    G = rng.standard_normal(len(ci))
    gC_ref, gT_ref = oracle.grad(lam, G, pattern_=(rp, ci))
    gC, gT = plan.adjoint(C, th, torch.tensor(G, device="cuda"))
    eG = max(_rel(gC.cpu().numpy(), gC_ref), _rel(gT.cpu().numpy(), gT_ref))
    uC_ref, uT_ref = oracle.grad_material(lam, oracle.grad_D_uu(lam, u))
    uC, uT = plan.adjoint_rank1(C, th, torch.tensor(u, device="cuda"))
    eU = max(_rel(uC.cpu().numpy(), uC_ref), _rel(uT.cpu().numpy(), uT_ref))
    print("  apply rel %.3e, adjoint rel %.3e, rank-one adjoint rel %.3e" % (ry, eG, eU), flush=True)
    assert ry <= TOL and eG <= GTOL and eU <= GTOL


@pytest.mark.parametrize("q", [3, 4])
def test_layerwise_wide_thickness_rows(oracle, L, q):
    """Rows of width q + 1 and 2q + 1 (7 or 9 at interfaces): the generic row
    body of the scatter, the adjoint streams for 7 and 9, the product."""
    lam = W.plate(2, 5, q, [0, 45, 90, -45], [W.material(W.CARBON), W.material(W.GLASS)], [0, 1, 1, 0], ne2=4,
                  name="layerwise_q%d" % q)
    print("case q=%d" % q, flush=True)
    ref = oracle.assemble(lam)
    for mode in ("bucket", "ply"):
        plan = _fast_full(oracle, L, lam, mode, ref=ref)
    _apply_and_adjoint(oracle, L, lam, plan, ref, np.random.default_rng(40 + q))


@pytest.mark.parametrize("seed", range(4))
def test_thickness_knot_inside_a_ply(oracle, L, seed):
    """One ply split into two thickness elements by an interior knot of random
    multiplicity (continuity C^{q-r} inside the ply), q drawn in 1..4."""
    rng = np.random.default_rng(4100 + seed)
    lam = W.random_small(rng, max_ply=4, n_mat=2, split_plies=True)
    print("case seed %d: p %d,%d q %d plies %d, thickness knots %s" % (seed, lam.p1, lam.p2, lam.q, lam.n_ply,
                                                                      np.round(lam.k3, 3).tolist()), flush=True)
    assert lam.nt > lam.q * lam.n_ply + 1  # more thickness functions than one element per ply gives
    ref = oracle.assemble(lam)
    _fast_full(oracle, L, lam, "bucket", ref=ref)
    plan = _fast_full(oracle, L, lam, "ply", ref=ref)
    _apply_and_adjoint(oracle, L, lam, plan, ref, rng)


@pytest.mark.parametrize("lds_kib", [0, 16])
def test_lds_mode_scatter(oracle, L, lds_kib):
    """One thickness element through all plies with nine harmonic sets per
    material: more than eight sets act on every thickness row, so the scatter
    runs in LDS mode.  With the default 80 KiB budget it stages P of the
    chunk's sets in LDS; with 16 KiB (8 KiB of it for the coefficients) not
    even one set's P fits next to a one-row tile, and P is read from memory."""
    rng = np.random.default_rng(4200 + lds_kib)
    lam = W.random_small(rng, paper_regime=True, max_ply=4, n_mat=1, p=2, q=2)
    print("case lds_kib %d plies %d" % (lds_kib, lam.n_ply), flush=True)
    _fast_full(oracle, L, lam, "harmonic9", tuning={"lds_kib": lds_kib} if lds_kib else None)


def _whole_plate(oracle, L, lam, mode, tuning=None):
    plan = L.Plan(lam, set_mode=mode, tuning=tuning)
    grp, gci = plan.pattern()
    C, th = _mats(lam)
    vals = plan.assemble(C, th)
    torch.cuda.synchronize()
    print("whole plate %s %s: nnz %d, oracle assembling" % (lam.name, mode, plan.nnz), flush=True)
    rp, ci, v = oracle.assemble(lam)
    assert np.array_equal(grp.cpu().numpy(), rp)
    del grp
    assert np.array_equal(gci.cpu().numpy(), ci)
    del gci, ci
    g = vals.cpu().numpy()
    del vals
    torch.cuda.empty_cache()
    relF = float(np.linalg.norm(g - v) / np.linalg.norm(v))
    relM = _rel(g, v)
    print("  relF %.3e relmax %.3e" % (relF, relM), flush=True)
    assert relF <= TOL and relM <= TOL


@pytest.mark.timeout(300)
def test_whole_matrix_p2_64x64_32ply(oracle, L):
    """Every one of the 242,809,488 nonzeros against the oracle's full assembly."""
    from paper_1905_05417_amd import autotune
    lam = W.config_p2_64x64_32ply()
    _whole_plate(oracle, L, lam, "bucket", autotune.lookup(lam, "bucket"))


@pytest.mark.timeout(600)
def test_whole_matrix_adjoint_plate_64ply(oracle, L):
    """Every one of the 1,081,559,952 nonzeros of the 64-ply plate (one set per
    ply, 4 materials, seeded angles) against the oracle's full assembly."""
    from paper_1905_05417_amd import autotune
    lam = W.config_adjoint_p2_96x96_64ply()
    _whole_plate(oracle, L, lam, "ply", autotune.lookup(lam, "bucket"))
