"""The experiment's setting (Sec. 4): one element of degree p through the
whole thickness, all plies inside it, so every set acts on every thickness
pair.  Fast and standard GPU assembly against the CPU oracle, full matrices,
relative Frobenius error 1e-12."""
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


CASES = [(1, 3, 1, "0/90"), (1, 4, 6, "0/90"), (2, 3, 2, "0/45/-45/90"), (2, 4, 9, "0/90"),
         (3, 2, 5, "0/45/-45/90"), (3, 3, 16, "0/90"), (4, 2, 3, "0/90"), (4, 2, 8, "0/45/-45/90")]


@pytest.mark.parametrize("p,ne,m,layup", CASES)
def test_paper_regime_fast_and_standard(oracle, L, p, ne, m, layup):
    lam = W.paper_plate(p, ne, m, layup)
    print("case", lam.name, flush=True)
    rp, ci, ref = oracle.assemble(lam)
    plan = L.Plan(lam, set_mode="bucket")
    rowptr, colind = plan.pattern()
    assert np.array_equal(rowptr.cpu().numpy(), rp) and np.array_equal(colind.cpu().numpy(), ci)
    C = torch.tensor(np.asarray(lam.C), device="cuda")
    th = torch.tensor(np.asarray(lam.theta), device="cuda")
    v = plan.assemble(C, th).cpu().numpy()
    err = float(np.linalg.norm(v - ref) / np.linalg.norm(ref))
    print("  fast rel %.2e" % err, flush=True)
    assert err <= TOL
    if p <= 3:  # the standard kernel keeps a cell's gradient table in LDS (p = 4 exceeds it)
        vs = plan.assemble_standard(C, th).cpu().numpy()
        err = float(np.linalg.norm(vs - ref) / np.linalg.norm(ref))
        print("  standard rel %.2e" % err, flush=True)
        assert err <= TOL
