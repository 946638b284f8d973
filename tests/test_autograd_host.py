"""The differentiable assembly's torch.autograd.Function on the CPU.

_Assemble only routes tensors: its forward calls plan.assemble and its
backward plan.adjoint.  Here a stand-in plan computes both with the CPU oracle
(the standard assembly of Sec. 2.4 and the gradient of L = <G, vals> through
every ply's rotated tensor), so the Function's own plumbing (shapes, views,
detaching, the refusal of bucket plans, the harmonic5 check) is checked by
torch.autograd.gradcheck without a GPU.  The GPU path behind the same
Function is tested in test_gpu_adjoint.py and test_gpu_setmodes.py.
"""
import copy

import numpy as np
import pytest
import torch

from paper_1905_05417_amd import lamasm
from paper_1905_05417_amd import workloads as W


class OraclePlan:
    """Duck-typed plan: assemble and adjoint from the oracle, on CPU tensors."""

    def __init__(self, oracle, lam, set_mode="ply"):
        self.o, self.lam, self.set_mode = oracle, lam, set_mode
        self.pat = oracle.pattern(lam)
        self.n_mat, self.n_ply = np.asarray(lam.C).shape[0], lam.n_ply
        self.checks = 0

    def _lam(self, C, theta):
        lam = copy.copy(self.lam)
        lam.C = C.reshape(self.n_mat, 6, 6).numpy().copy()
        lam.theta = theta.numpy().copy()
        return lam

    def assemble(self, C, theta):
        return torch.from_numpy(self.o.assemble(self._lam(C, theta), pattern_=self.pat)[2])

    def adjoint(self, C, theta, grad_vals):
        gC, gT = self.o.grad(self._lam(C, theta), grad_vals.detach().numpy(), pattern_=self.pat)
        return torch.from_numpy(gC), torch.from_numpy(gT)

    def check(self):
        self.checks += 1


def _small(seed):
    rng = np.random.default_rng(seed)
    lam = W.random_small(rng, p=1, q=1, max_ply=3, n_mat=2)
    return lam


def test_gradcheck_through_oracle_plan(oracle):
    lam = _small(3)
    plan = OraclePlan(oracle, lam)
    C = torch.tensor(np.asarray(lam.C), dtype=torch.float64, requires_grad=True)
    th = torch.tensor(np.asarray(lam.theta), dtype=torch.float64, requires_grad=True)
    G = torch.from_numpy(np.random.default_rng(1).standard_normal(len(plan.pat[1])))

    def f(C_, th_):
        return (lamasm._Assemble.apply(C_, th_, plan) * G).sum()

    assert torch.autograd.gradcheck(f, (C, th), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_backward_shapes_and_values(oracle):
    lam = _small(4)
    plan = OraclePlan(oracle, lam)
    C = torch.tensor(np.asarray(lam.C), dtype=torch.float64, requires_grad=True)
    th = torch.tensor(np.asarray(lam.theta), dtype=torch.float64, requires_grad=True)
    G = np.random.default_rng(2).standard_normal(len(plan.pat[1]))
    vals = lamasm.assemble(plan, C, th)
    assert vals.shape == (len(plan.pat[1]),) and vals.requires_grad
    (vals * torch.from_numpy(G)).sum().backward()
    gC_ref, gT_ref = oracle.grad(lam, G, pattern_=plan.pat)
    assert C.grad.shape == C.shape and th.grad.shape == th.shape
    assert np.allclose(C.grad.numpy(), gC_ref, rtol=0, atol=1e-12 * np.abs(gC_ref).max())
    assert np.allclose(th.grad.numpy(), gT_ref, rtol=0, atol=1e-12 * np.abs(gT_ref).max())


def test_bucket_plans_are_refused(oracle):
    lam = _small(5)
    plan = OraclePlan(oracle, lam, set_mode="bucket")
    C = torch.tensor(np.asarray(lam.C), dtype=torch.float64, requires_grad=True)
    th = torch.tensor(np.asarray(lam.theta), dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError, match="bucket"):
        lamasm.assemble(plan, C, th)


def test_harmonic5_forward_checks_the_device_flags(oracle):
    lam = _small(6)
    plan = OraclePlan(oracle, lam, set_mode="harmonic5")
    C = torch.tensor(np.asarray(lam.C), dtype=torch.float64, requires_grad=True)
    th = torch.tensor(np.asarray(lam.theta), dtype=torch.float64, requires_grad=True)
    lamasm.assemble(plan, C, th)
    assert plan.checks == 1
    plan9 = OraclePlan(oracle, lam, set_mode="harmonic9")
    lamasm.assemble(plan9, C, th)
    assert plan9.checks == 0


def test_default_set_mode_is_per_ply():
    assert lamasm.default_set_mode(W.config_q1_8x8()) == "ply"
