"""Set modes against per-ply angle changes (Sec. 3: one 2D operator per set of
plies sharing material and orientation; Remark on orientations: harmonic
sets for arbitrary angles).

A plan fixes its sets when it is created; the angles are passed at every
assembly.  'ply' and the harmonic modes must give K(theta) for any theta
(element by element against the CPU oracle, relative Frobenius <= 1e-12);
a bucket plan given angles that differ inside one of its sets, and a
harmonic5 plan given a material whose rotation has odd harmonics, must raise
their status flag (lam_check) instead of passing silently.
"""
import copy

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


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _full_parity(oracle, plan, lam, vals):
    rp, ci, ref = oracle.assemble(lam)
    rowptr, colind = plan.pattern()
    assert np.array_equal(rowptr.cpu().numpy(), rp) and np.array_equal(colind.cpu().numpy(), ci)
    got = vals.cpu().numpy()
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("mode", ["ply", "harmonic9", "harmonic5"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_single_ply_angle_change(oracle, L, mode, seed):
    """Plan made at the original angles, assembled at angles where one ply moved."""
    rng = np.random.default_rng(700 + seed)
    lam = W.random_small(rng, max_ply=6, n_mat=2, anisotropic=(mode != "harmonic5"))
    plan = L.Plan(lam, set_mode=mode)
    moved = copy.copy(lam)
    moved.theta = np.array(lam.theta, dtype=np.float64)
    j = int(rng.integers(0, lam.n_ply))
    moved.theta[j] += 0.7
    print("mode %s seed %d plies %d moved ply %d" % (mode, seed, lam.n_ply, j), flush=True)
    vals = plan.assemble(_dev(lam.C), _dev(moved.theta))
    plan.check()
    rel = _full_parity(oracle, plan, moved, vals)
    print("  rel %.3e" % rel, flush=True)
    assert rel <= TOL


def _bucket_plate():
    # [0/90/0/90/0] carbon, two bucket sets of 3 and 2 plies
    return W.plate(2, 3, 2, [0, 90, 0, 90, 0], [W.material(W.CARBON)], [0] * 5, ne2=2, name="bucket5")


def test_bucket_disagreement_is_flagged(oracle, L):
    lam = _bucket_plate()
    plan = L.Plan(lam, set_mode="bucket")
    assert plan.n_sets == 2
    C = _dev(lam.C)
    th = np.array(lam.theta)
    plan.assemble(C, _dev(th))
    plan.check()  # the plan-time angles agree within every set
    bad = th.copy()
    bad[2] += 0.1  # ply 2 leaves the set of plies 0 and 4
    plan.assemble(C, _dev(bad))
    with pytest.raises(ValueError, match="bucket set"):
        plan.check()
    plan.check()  # the flag was cleared by the failed check
    # a whole set turned together stays one orientation: exact
    turned = copy.copy(lam)
    turned.theta = th.copy()
    turned.theta[[0, 2, 4]] += 0.3
    vals = plan.assemble(C, _dev(turned.theta))
    plan.check()
    assert _full_parity(oracle, plan, turned, vals) <= TOL


def test_harmonic5_coupled_material_is_flagged(L):
    rng = np.random.default_rng(710)
    lam = W.random_small(rng, max_ply=3, n_mat=1, anisotropic=True)
    plan = L.Plan(lam, set_mode="harmonic5")
    plan.assemble(_dev(lam.C), _dev(lam.theta))
    with pytest.raises(ValueError, match="harmonic5"):
        plan.check()
    # the same material through nine harmonics: no flag
    plan9 = L.Plan(lam, set_mode="harmonic9")
    plan9.assemble(_dev(lam.C), _dev(lam.theta))
    plan9.check()


def _quad(plan, vals, rowptr, colind, u):
    rows = torch.repeat_interleave(torch.arange(plan.n_rows, device="cuda"), rowptr[1:] - rowptr[:-1])
    return float((u[rows] * vals * u[colind.long()]).sum())


def test_default_plan_adjoint_vs_central_differences(oracle, L):
    """The default plan ('ply' sets): dL/dtheta of L = u^T K u by the adjoint
    against central differences of the forward, one ply angle at a time,
    and against the oracle's gradient."""
    rng = np.random.default_rng(720)
    lam = W.plate(2, 6, 2, list(rng.uniform(0, 180, 5)), [W.material(W.CARBON), W.material(W.GLASS)],
                  [0, 1, 0, 1, 1], ne2=5, name="fd_default")
    plan = L.Plan(lam)
    assert plan.set_mode == "ply"
    rowptr, colind = plan.pattern()
    C, th = _dev(lam.C), _dev(lam.theta)
    u = torch.tensor(rng.standard_normal(plan.n_rows), device="cuda")
    gC, gT = plan.adjoint_rank1(C, th, u)
    gT = gT.cpu().numpy()
    h = 1e-6
    worst = 0.0
    for l in range(lam.n_ply):
        tp, tm = th.clone(), th.clone()
        tp[l] += h
        tm[l] -= h
        fd = (_quad(plan, plan.assemble(C, tp), rowptr, colind, u) -
              _quad(plan, plan.assemble(C, tm), rowptr, colind, u)) / (2 * h)
        worst = max(worst, abs(fd - gT[l]) / np.abs(gT).max())
    plan.check()
    gC_ref, gT_ref = oracle.grad_material(lam, oracle.grad_D_uu(lam, u.cpu().numpy()))
    e_or = max(float(np.abs(gT - gT_ref).max() / np.abs(gT_ref).max()),
               float(np.abs(gC.cpu().numpy() - gC_ref).max() / np.abs(gC_ref).max()))
    print("FD worst %.3e, vs oracle %.3e" % (worst, e_or), flush=True)
    assert worst <= 1e-7 and e_or <= 1e-10
