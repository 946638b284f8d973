"""Pins of the oracle's building blocks: quadrature, B-splines, ply rotation.

Each test compares the oracle with something other than itself: a library
routine (numpy's Gauss-Legendre, scipy's B-splines), a closed form (moments of
polynomials, the classical laminate transformation formulas derived from the
strain energy), or an invariant of the mathematics.
"""
import numpy as np
import pytest

from paper_1905_05417_amd import workloads as W


# ----------------------------------------------------------- quadrature ----
@pytest.mark.parametrize("n", list(range(1, 21)))
def test_gauss_matches_numpy(oracle, n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, rtol=0, atol=1e-15)
    assert np.allclose(w, wr, rtol=0, atol=4e-15)  # both rules carry a few ulps of rounding


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_gauss_exact_on_monomials(oracle, n):
    x, w = oracle.gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14
    # and not exact one degree higher (so the rule really has n points)
    k = 2 * n
    assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-8


# ------------------------------------------------------------- B-splines ----
def _random_open_knots(rng, p, ne, repeat=True):
    inner = np.sort(rng.uniform(0.02, 0.98, size=ne - 1))
    if repeat and ne >= 3 and p >= 2:
        inner = np.sort(np.concatenate([inner, inner[1:2]]))
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_bspline_matches_scipy(oracle, p):
    from scipy.interpolate import BSpline
    rng = np.random.default_rng(100 + p)
    for trial in range(4):
        t = _random_open_knots(rng, p, int(rng.integers(1, 6)), repeat=(trial % 2 == 0))
        n = len(t) - p - 1
        spl = BSpline(t, np.eye(n), p, extrapolate=False)
        dspl = spl.derivative() if p > 0 else None
        for x in rng.uniform(0, 1, size=25):
            if np.any(np.isclose(x, t)):
                continue
            N, dN = oracle.bspline_eval(p, t, x)
            assert np.allclose(N, spl(x), rtol=0, atol=1e-13)
            if p > 0:
                assert np.allclose(dN, dspl(x), rtol=0, atol=1e-10 * max(1.0, np.abs(dspl(x)).max()))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_bspline_partition_and_linear_precision(oracle, p):
    rng = np.random.default_rng(7 + p)
    t = _random_open_knots(rng, p, 5)
    g = W.greville(p, t)
    for x in np.concatenate([rng.uniform(0, 1, 20), [0.0, 1.0]]):
        N, dN = oracle.bspline_eval(p, t, x)
        assert abs(N.sum() - 1.0) < 1e-14
        assert abs(dN.sum()) < 1e-11
        assert abs(np.dot(g, N) - x) < 1e-14
        assert abs(np.dot(g, dN) - 1.0) < 1e-11


# ------------------------------------------------------------- rotation ----
def _ortho(rng):
    return W.material(W.jittered(W.CARBON, rng))


def test_rotation_identity(oracle):
    rng = np.random.default_rng(1)
    C = W.random_anisotropic(rng)
    assert np.allclose(oracle.rotate(C, 0.0), C, rtol=0, atol=1e-13)


def test_rotation_inplane_block_textbook(oracle):
    """In-plane block of an orthotropic ply rotated by theta (fibre at angle
    theta from x, counterclockwise): the classical transformed-stiffness
    formulas (Q-bar_11 ... Q-bar_66).  Our Voigt index 3 is the 12 shear."""
    rng = np.random.default_rng(2)
    C = _ortho(rng)
    Q11, Q12, Q22, Q66 = C[0, 0], C[0, 1], C[1, 1], C[3, 3]
    for th in rng.uniform(-np.pi, np.pi, size=6):
        c, s = np.cos(th), np.sin(th)
        D = oracle.rotate(C, th)
        ref = {
            (0, 0): Q11 * c**4 + 2 * (Q12 + 2 * Q66) * s**2 * c**2 + Q22 * s**4,
            (0, 1): (Q11 + Q22 - 4 * Q66) * s**2 * c**2 + Q12 * (s**4 + c**4),
            (1, 1): Q11 * s**4 + 2 * (Q12 + 2 * Q66) * s**2 * c**2 + Q22 * c**4,
            (0, 3): (Q11 - Q12 - 2 * Q66) * s * c**3 + (Q12 - Q22 + 2 * Q66) * s**3 * c,
            (1, 3): (Q11 - Q12 - 2 * Q66) * s**3 * c + (Q12 - Q22 + 2 * Q66) * s * c**3,
            (3, 3): (Q11 + Q22 - 2 * Q12 - 2 * Q66) * s**2 * c**2 + Q66 * (s**4 + c**4),
        }
        for (i, j), v in ref.items():
            assert abs(D[i, j] - v) < 1e-12 * abs(C).max(), (i, j)
            assert abs(D[j, i] - v) < 1e-12 * abs(C).max(), (j, i)


def test_rotation_out_of_plane_blocks_from_energy(oracle):
    """Transverse shear and 33 couplings, from the strain energy: with material
    strains gamma_1z = c g_xz + s g_yz, gamma_2z = -s g_xz + c g_yz and
    eps_11 = c^2 e_xx + s^2 e_yy + cs g_xy, eps_22 = s^2 e_xx + c^2 e_yy - cs g_xy."""
    rng = np.random.default_rng(3)
    C = _ortho(rng)
    for th in rng.uniform(-np.pi, np.pi, size=5):
        c, s = np.cos(th), np.sin(th)
        D = oracle.rotate(C, th)
        G13, G23 = C[4, 4], C[5, 5]
        tol = 1e-12 * abs(C).max()
        assert abs(D[4, 4] - (G13 * c * c + G23 * s * s)) < tol
        assert abs(D[5, 5] - (G13 * s * s + G23 * c * c)) < tol
        assert abs(D[4, 5] - (G13 - G23) * c * s) < tol
        assert abs(D[0, 2] - (C[0, 2] * c * c + C[1, 2] * s * s)) < tol
        assert abs(D[1, 2] - (C[0, 2] * s * s + C[1, 2] * c * c)) < tol
        assert abs(D[2, 3] - (C[0, 2] - C[1, 2]) * c * s) < tol
        assert abs(D[2, 2] - C[2, 2]) < tol
        # orthotropic about e3: no coupling between {11,22,33,12} and {13,23}
        assert np.abs(D[:4, 4:]).max() < tol


def _tensor(D):
    v = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4, (1, 2): 5, (2, 1): 5}
    T = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    T[i, j, k, l] = D[v[i, j], v[k, l]]
    return T


def test_rotation_invariants_and_composition(oracle):
    rng = np.random.default_rng(4)
    C = W.random_anisotropic(rng)
    T0 = _tensor(C)
    inv0 = (np.einsum("iijj", T0), np.einsum("ijij", T0), np.linalg.norm(T0))
    for th in rng.uniform(-np.pi, np.pi, size=4):
        T = _tensor(oracle.rotate(C, th))
        inv = (np.einsum("iijj", T), np.einsum("ijij", T), np.linalg.norm(T))
        assert np.allclose(inv, inv0, rtol=1e-13)
        a, b = rng.uniform(-3, 3, size=2)
        assert np.allclose(oracle.rotate(oracle.rotate(C, a), b), oracle.rotate(C, a + b), rtol=0,
                           atol=1e-12 * abs(C).max())
    # a half turn is diag(-1,-1,1): components with an odd count of in-plane
    # indices flip sign, i.e. D(pi) = S C S with S = diag(1,1,1,1,-1,-1)
    S = np.diag([1.0, 1, 1, 1, -1, -1])
    assert np.allclose(oracle.rotate(C, np.pi), S @ C @ S, rtol=0, atol=1e-12 * abs(C).max())


def test_isotropic_is_rotation_invariant(oracle):
    C = W.isotropic(70.0, 0.3)
    for th in (0.3, 1.1, 2.9):
        assert np.allclose(oracle.rotate(C, th), C, rtol=0, atol=1e-12 * abs(C).max())


def test_rotation_derivative_vs_central_difference(oracle):
    rng = np.random.default_rng(5)
    C = W.random_anisotropic(rng)
    h = 1e-5
    for th in rng.uniform(-np.pi, np.pi, size=4):
        fd = (oracle.rotate(C, th + h) - oracle.rotate(C, th - h)) / (2 * h)
        assert np.allclose(oracle.rotate_dtheta(C, th), fd, rtol=0, atol=1e-8 * abs(C).max())


def test_harmonic_content(oracle):
    """D(theta) is a trigonometric polynomial of degree 4 for any 6x6; only even
    harmonics {1, cos2t, sin2t, cos4t, sin4t} for an orthotropic ply, which is
    the span of the five-term split of Remark 3 (1, c^4, c^3 s, c^2, c s)."""
    rng = np.random.default_rng(6)
    Ca = W.random_anisotropic(rng)
    N = 9
    ts = 2 * np.pi * np.arange(N) / N
    Ds = np.stack([oracle.rotate(Ca, t) for t in ts])
    coef = np.fft.rfft(Ds, axis=0) / N  # harmonics 0..4
    for th in rng.uniform(-np.pi, np.pi, size=4):
        rec = coef[0].real + sum(2 * (coef[k] * np.exp(1j * k * th)).real for k in range(1, 5))
        assert np.allclose(rec, oracle.rotate(Ca, th), rtol=0, atol=1e-12 * abs(Ca).max())
    # the general case really has odd harmonics (so a five-term split is not enough)
    assert np.abs(coef[1]).max() > 1e-3 * abs(Ca).max()

    Co = _ortho(rng)
    basis = lambda t: np.array([1.0, np.cos(t) ** 4, np.cos(t) ** 3 * np.sin(t), np.cos(t) ** 2,
                                np.cos(t) * np.sin(t)])
    fit_t = np.array([0.1, 0.5, 0.9, 1.7, 2.6])
    Phi = np.stack([basis(t) for t in fit_t])
    Dfit = np.stack([oracle.rotate(Co, t) for t in fit_t]).reshape(5, 36)
    A = np.linalg.solve(Phi, Dfit)
    for th in rng.uniform(-np.pi, np.pi, size=6):
        assert np.allclose(basis(th) @ A, oracle.rotate(Co, th).reshape(36), rtol=0, atol=1e-10 * abs(Co).max())
