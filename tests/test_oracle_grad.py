"""Pins of the oracle's gradient of L = <G, K> (material moduli and ply angles).

Independent checks: central finite differences of L computed with the pinned
assembly (compensated sums), Euler's identity for a function linear in C, the
closed form dL/dD_l = V_l eps eps^T for a linear displacement field with
G = u u^T, and the vanishing angle gradient for isotropic plies.
"""
import math

import numpy as np
import pytest

from paper_1905_05417_amd import workloads as W


def _L(oracle, lam, G, pat):
    _, _, v = oracle.assemble(lam, pattern_=pat)
    return math.fsum(G * v)


def _G_uu(lam, pat, u):
    rp, ci = pat
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return u[rows] * u[ci]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_vs_central_differences(oracle, seed):
    rng = np.random.default_rng(seed)
    lam = W.random_small(rng, paper_regime=(seed == 2), max_ply=3)
    pat = oracle.pattern(lam)
    u = rng.standard_normal(lam.n_rows)
    G = _G_uu(lam, pat, u)
    gC, gT = oracle.grad(lam, G, pattern_=pat)
    h = 1e-6
    scale_T = max(np.abs(gT).max(), 1e-300)
    for l in range(lam.n_ply):
        th0 = lam.theta[l]
        lam.theta[l] = th0 + h
        Lp = _L(oracle, lam, G, pat)
        lam.theta[l] = th0 - h
        Lm = _L(oracle, lam, G, pat)
        lam.theta[l] = th0
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gT[l]) < 1e-7 * scale_T, (l, fd, gT[l])
    scale_C = np.abs(gC).max()
    for (m, a, b) in [(0, 0, 0), (0, 1, 4), (lam.C.shape[0] - 1, 5, 3), (0, 3, 3), (0, 2, 1)]:
        c0 = lam.C[m, a, b]
        hc = 1e-6 * max(abs(c0), 1.0)
        lam.C[m, a, b] = c0 + hc
        Lp = _L(oracle, lam, G, pat)
        lam.C[m, a, b] = c0 - hc
        Lm = _L(oracle, lam, G, pat)
        lam.C[m, a, b] = c0
        fd = (Lp - Lm) / (2 * hc)
        assert abs(fd - gC[m, a, b]) < 1e-7 * scale_C, (m, a, b, fd, gC[m, a, b])


def test_euler_identity(oracle):
    """L is linear in every C_m, so sum_m <C_m, dL/dC_m> = L exactly."""
    rng = np.random.default_rng(4)
    lam = W.random_small(rng, max_ply=4, n_mat=3)
    pat = oracle.pattern(lam)
    G = rng.standard_normal(len(pat[1]))
    gC, _ = oracle.grad(lam, G, pattern_=pat)
    L = _L(oracle, lam, G, pat)
    assert abs(math.fsum((lam.C * gC).ravel()) - L) < 1e-12 * max(abs(L), np.abs(G).max())


def test_linear_field_closed_form(oracle):
    """For u = A x + b and G = u u^T, dL/dD_l = V_l eps eps^T (V_l the ply
    volume), hence dL/dtheta_l = V_l eps^T dD/dtheta eps."""
    rng = np.random.default_rng(5)
    lam = W.random_small(rng, max_ply=3)
    pat = oracle.pattern(lam)
    X = W.control_points(lam)
    A = rng.standard_normal((3, 3))
    u = (X @ A.T + rng.standard_normal(3)).ravel()
    G = _G_uu(lam, pat, u)
    dD = oracle.grad_D(lam, pat[0], pat[1], G)
    eps = np.array([A[0, 0], A[1, 1], A[2, 2], A[0, 1] + A[1, 0], A[0, 2] + A[2, 0], A[1, 2] + A[2, 1]])
    V = abs(np.linalg.det(lam.jac)) * np.diff(lam.iface)
    for l in range(lam.n_ply):
        ref = V[l] * np.outer(eps, eps)
        assert np.abs(dD[l] - ref).max() < 1e-12 * np.abs(ref).max()
    _, gT = oracle.grad_material(lam, dD)
    for l in range(lam.n_ply):
        ref = V[l] * eps @ oracle.rotate_dtheta(lam.C[lam.ply_mat[l]], lam.theta[l]) @ eps
        assert abs(gT[l] - ref) < 1e-11 * max(abs(ref), 1.0)


def test_isotropic_angle_gradient_is_zero(oracle):
    rng = np.random.default_rng(6)
    lam = W.random_small(rng, max_ply=3, n_mat=1)
    lam.C = np.stack([W.isotropic(30.0, 0.2)])
    pat = oracle.pattern(lam)
    G = rng.standard_normal(len(pat[1]))
    gC, gT = oracle.grad(lam, G, pattern_=pat)
    assert np.abs(gT).max() < 1e-12 * np.abs(gC).max() * np.abs(lam.C).max()


def test_uu_gradient_equals_general_gradient(oracle):
    """The u u^T specialisation (used at full size) agrees with the general
    gradient fed G = u u^T, and with u^T K u's Euler identity."""
    rng = np.random.default_rng(7)
    for k in range(3):
        lam = W.random_small(rng, paper_regime=(k == 1), max_ply=3)
        pat = oracle.pattern(lam)
        u = rng.standard_normal(lam.n_rows)
        dD = oracle.grad_D(lam, pat[0], pat[1], _G_uu(lam, pat, u))
        dU = oracle.grad_D_uu(lam, u)
        assert np.abs(dD - dU).max() < 1e-12 * np.abs(dD).max()
        _, _, v = oracle.assemble(lam, pattern_=pat)
        L = math.fsum(_G_uu(lam, pat, u) * v)
        Ds = np.stack([oracle.rotate(lam.C[lam.ply_mat[l]], lam.theta[l]) for l in range(lam.n_ply)])
        assert abs(math.fsum((Ds * dU).ravel()) - L) < 1e-12 * abs(L)
