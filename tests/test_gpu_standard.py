"""GPU parity of the standard 3D element-by-element assembly (the comparator of
the method) against the CPU oracle, and fast vs standard on the same CSR.

The cases reach both element kernels: one ply cell per element with at most
eight 16-wide tile pairs of local functions (the block-per-element kernel with
the gradient table in LDS: degrees 1-3 layerwise) and the wavefront-per-pair
kernel (degree 4, and one element through several plies)."""
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


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("case", range(9))
def test_standard_matches_oracle(oracle, L, case):
    """Cases 6-8 are degree 4 (the gradient table of all points exceeds the
    LDS budget: the kernel takes the points in chunks), in layerwise and
    one-element-through-the-thickness spaces."""
    rng = np.random.default_rng(3000 + case)
    if case == 0:
        lam = W.config_q1_8x8()
    elif case == 1:
        lam = W.plate(2, 5, 2, [0, 45, 90], [W.material(W.CARBON), W.material(W.GLASS)], [0, 1, 0], ne2=4)
    elif case == 6:
        lam = W.plate(4, 3, 2, [0, 45, 90], [W.material(W.CARBON), W.material(W.GLASS)], [0, 1, 0], ne2=2)
    elif case == 7:
        lam = W.paper_plate(4, 2, 3, "0/45/-45/90")
    elif case == 8:
        lam = W.random_small(rng, p=4, q=4, max_ply=3)
    else:
        lam = W.random_small(rng, paper_regime=(case % 2 == 1), max_ply=4)
    print("case", case, lam.p1, lam.p2, lam.q, lam.n_ply, flush=True)
    rp, ci, v = oracle.assemble(lam)
    plan = L.Plan(lam, set_mode="bucket")
    C, th = _mats(lam)
    vs = plan.assemble_standard(C, th).cpu().numpy()
    vf = plan.assemble(C, th).cpu().numpy()
    rf, rm = _rel(vs, v)
    print("  standard vs oracle relF %.3e relmax %.3e" % (rf, rm), flush=True)
    assert rf <= TOL and rm <= TOL
    rf, rm = _rel(vf, vs)
    print("  fast vs standard relF %.3e relmax %.3e" % (rf, rm), flush=True)
    assert rf <= TOL and rm <= TOL


def test_standard_full_size_p2_64x64_32ply(L):
    """Fast and standard agree on the whole 243M-nonzero CSR."""
    lam = W.config_p2_64x64_32ply()
    plan = L.Plan(lam, set_mode="bucket")
    C, th = _mats(lam)
    vf = plan.assemble(C, th)
    vs = plan.assemble_standard(C, th)
    d = torch.linalg.vector_norm(vf - vs) / torch.linalg.vector_norm(vs)
    m = (vf - vs).abs().max() / vs.abs().max()
    print("fast vs standard relF %.3e relmax %.3e" % (float(d), float(m)), flush=True)
    assert float(d) <= TOL and float(m) <= TOL
    vs2 = plan.assemble_standard(C, th)
    assert torch.equal(vs, vs2), "standard assembly is not deterministic"
