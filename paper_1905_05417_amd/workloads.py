"""Seeded synthetic laminates (inputs only; no assembly arithmetic here).

Both the GPU path and the CPU oracle are fed from this module and nothing
else is shared between them.  A `Laminate` carries everything the operator
needs: open knot vectors (in-plane degrees p1, p2, thickness degree q), the
constant map gradient of the extruded box, the ply stack and the materials.

Workloads mirror the paper's setting (Sec. 4: flat plate, tensor-product
B-splines in-plane, plies stacked [0/90]... or [0/45/-45/90]..., orthotropic
plies rotated about the plate normal), at the sizes used by the tests and the
benchmark.  Readings fixed here (the paper leaves them open):
  * thickness space: degree q per ply, one element per ply, C0 at interfaces
    (interior interface knots repeated q times);
  * total laminate thickness H (0.1 for the Q1 case, 0.02 otherwise), plies of
    equal thickness, ply 0 at the bottom;
  * angles are counterclockwise about +e3, fibre axis (cos t, sin t, 0);
  * engineering constants -> 6x6 by inverting the compliance in Voigt order
    (11,22,33,12,13,23) with engineering shears.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BATCH = 190505417
SEED_ADJOINT = 190505418
SEED_U = 190505419


@dataclass
class Laminate:
    p1: int
    k1: np.ndarray
    p2: int
    k2: np.ndarray
    q: int
    k3: np.ndarray
    jac: np.ndarray            # (3,3) DF, constant
    iface: np.ndarray          # (n_ply+1,)
    ply_mat: np.ndarray        # (n_ply,) int32
    theta: np.ndarray          # (n_ply,) radians
    C: np.ndarray              # (n_mat,6,6) material axes
    ng: tuple = (0, 0, 0)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n1(self):
        return len(self.k1) - self.p1 - 1

    @property
    def n2(self):
        return len(self.k2) - self.p2 - 1

    @property
    def nt(self):
        return len(self.k3) - self.q - 1

    @property
    def n_ply(self):
        return len(self.theta)

    @property
    def n_rows(self):
        return 3 * self.n1 * self.n2 * self.nt


# ---------------------------------------------------------------- knots ----
def open_uniform_knots(p: int, ne: int) -> np.ndarray:
    """C^{p-1} open uniform knots on [0,1] with ne elements."""
    inner = np.arange(1, ne) / ne
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def layerwise_knots(q: int, iface: np.ndarray) -> np.ndarray:
    """Thickness knots: one element per ply, C0 at every interior interface."""
    inner = np.repeat(np.asarray(iface[1:-1], dtype=np.float64), q)
    return np.concatenate([np.zeros(q + 1), inner, np.ones(q + 1)])


def uniform_iface(m: int) -> np.ndarray:
    return np.arange(m + 1) / m


def box_jac(Lx: float, Ly: float, H: float) -> np.ndarray:
    return np.diag([Lx, Ly, H]).astype(np.float64)


# ------------------------------------------------------------ materials ----
def orthotropic(E1, E2, E3, G12, G13, G23, nu12, nu13, nu23) -> np.ndarray:
    S = np.zeros((6, 6))
    S[0, 0], S[1, 1], S[2, 2] = 1 / E1, 1 / E2, 1 / E3
    S[0, 1] = S[1, 0] = -nu12 / E1
    S[0, 2] = S[2, 0] = -nu13 / E1
    S[1, 2] = S[2, 1] = -nu23 / E2
    S[3, 3], S[4, 4], S[5, 5] = 1 / G12, 1 / G13, 1 / G23
    return np.linalg.inv(S)


def isotropic(E, nu) -> np.ndarray:
    G = E / (2 * (1 + nu))
    return orthotropic(E, E, E, G, G, G, nu, nu, nu)


CARBON = dict(E1=175.0, E2=7.0, E3=7.0, G12=3.5, G13=3.5, G23=1.4, nu12=0.25, nu13=0.25, nu23=0.25)
GLASS = dict(E1=45.0, E2=12.0, E3=12.0, G12=5.5, G13=5.5, G23=4.5, nu12=0.28, nu13=0.28, nu23=0.28)
PAGANO = dict(E1=25.0, E2=1.0, E3=1.0, G12=0.2, G13=0.2, G23=0.5, nu12=0.25, nu13=0.25, nu23=0.25)


def material(d: dict) -> np.ndarray:
    return orthotropic(**d)


def jittered(d: dict, rng: np.random.Generator, lo=0.8, hi=1.2) -> dict:
    out = dict(d)
    for k in ("E1", "E2", "E3", "G12", "G13", "G23"):
        out[k] = d[k] * rng.uniform(lo, hi)
    return out


def random_anisotropic(rng: np.random.Generator, scale=10.0) -> np.ndarray:
    """A fully anisotropic symmetric positive definite 6x6 (all 21 entries)."""
    A = rng.standard_normal((6, 6))
    return scale * (A @ A.T / 6.0 + np.eye(6))


def deg(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64) * (np.pi / 180.0)


# ------------------------------------------------------------ laminates ----
def plate(p, ne, q, angles_deg, mats, ply_mat, H=0.02, L=(1.0, 1.0), name="", ne2=None, p2=None):
    m = len(angles_deg)
    iface = uniform_iface(m)
    p2 = p if p2 is None else p2
    ne2 = ne if ne2 is None else ne2
    return Laminate(
        p1=p, k1=open_uniform_knots(p, ne), p2=p2, k2=open_uniform_knots(p2, ne2),
        q=q, k3=layerwise_knots(q, iface), jac=box_jac(L[0], L[1], H), iface=iface,
        ply_mat=np.asarray(ply_mat, dtype=np.int32), theta=deg(angles_deg),
        C=np.stack([np.asarray(c, dtype=np.float64) for c in mats]), name=name)


def paper_plate(p: int, ne: int, m: int, layup: str = "0/90", H: float = 0.02) -> Laminate:
    """The experiment's setting (Sec. 4): one element of degree p through the
    whole thickness (all m plies inside it), degree p C^{p-1} in-plane with
    ne x ne elements, m uniform plies of the Pagano-type orthotropic material
    (moduli as printed), layup 0/90/0/90... or 0/45/-45/90/...; Gauss rules
    p + 1 per direction per element and per ply."""
    pattern = {"0/90": [0.0, 90.0], "0/45/-45/90": [0.0, 45.0, -45.0, 90.0]}[layup]
    angles = [pattern[l % len(pattern)] for l in range(m)]
    lam = plate(p, ne, p, angles, [material(PAGANO)], [0] * m, H=H,
                name="paper_p%d_%dx%d_%dply_%s" % (p, ne, ne, m, layup.replace("/", "_")))
    lam.k3 = open_uniform_knots(p, 1)
    lam.ng = (p + 1, p + 1, p + 1)
    return lam


def config_q1_8x8() -> Laminate:
    """Trilinear Q1 hexahedra, 8x8 in-plane, 4 plies [0/90/0/90] 1 element each,
    1x1x0.1 plate, carbon, 2x2x2 Gauss: 1215 DOF."""
    lam = plate(1, 8, 1, [0, 90, 0, 90], [material(CARBON)], [0] * 4, H=0.1, name="q1_8x8_4ply")
    lam.ng = (2, 2, 2)
    return lam


def config_p2_64x64_32ply() -> Laminate:
    """Degree-2 C1 B-splines 64x64 in-plane, 32 plies [0/90]_16 carbon, degree 2
    per ply (C0 interfaces), thickness 0.02, 3x3x3 Gauss: 849,420 DOF."""
    lam = plate(2, 64, 2, [0, 90] * 16, [material(CARBON)], [0] * 32, name="p2_64x64_32ply")
    lam.ng = (3, 3, 3)
    return lam


def config_p3_128x128_128ply() -> Laminate:
    """Degree-3 in-plane 128x128, 128 plies [0/45/-45/90]_32, carbon and glass
    alternating every 16 plies, degree 2 per ply."""
    angles = [0, 45, -45, 90] * 32
    ply_mat = [(l // 16) % 2 for l in range(128)]
    lam = plate(3, 128, 2, angles, [material(CARBON), material(GLASS)], ply_mat, name="p3_128x128_128ply")
    lam.ng = (4, 4, 3)
    return lam


def config_adjoint_p2_96x96_64ply(seed=SEED_ADJOINT) -> Laminate:
    """Degree 2, 96x96 in-plane, 64 plies with uniform random angles in [0,180)
    degrees and 4 materials (carbon, glass, and a +-20% modulus jitter of each)."""
    rng = np.random.default_rng(seed)
    mats = [material(CARBON), material(GLASS), material(jittered(CARBON, rng)), material(jittered(GLASS, rng))]
    ply_mat = rng.integers(0, 4, size=64)
    angles = rng.uniform(0.0, 180.0, size=64)
    lam = plate(2, 96, 2, angles, mats, ply_mat, name="adjoint_p2_96x96_64ply")
    lam.ng = (3, 3, 3)
    return lam


def batch_laminates(n=256, seed=SEED_BATCH):
    """Uneven laminates: in-plane elements 16..96 per side (each side drawn),
    degree 2..3, 4..64 plies; per laminate, with probability 0.7 every ply angle
    is drawn from {0,45,-45,90}, otherwise uniform in [0,180); one carbon-based
    material with +-20% modulus jitter."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        nx, ny = (int(v) for v in rng.integers(16, 97, size=2))
        p = int(rng.integers(2, 4))
        m = int(rng.integers(4, 65))
        if rng.uniform() < 0.7:
            angles = rng.choice([0.0, 45.0, -45.0, 90.0], size=m)
        else:
            angles = rng.uniform(0.0, 180.0, size=m)
        mat = material(jittered(CARBON, rng))
        lam = plate(p, nx, 2, angles, [mat], [0] * m, name="batch%03d" % b, ne2=ny)
        out.append(lam)
    return out


def random_small(rng: np.random.Generator, p=None, q=None, paper_regime=False, anisotropic=True, sheared=True,
                 n_mat=2, max_ply=4, split_plies=None) -> Laminate:
    """A tiny laminate with nonuniform knots (one repeated interior knot),
    a sheared affine map, fully anisotropic materials and random angles;
    in-plane degrees 1..3, thickness degree 1..4.  paper_regime: one
    thickness element spanning all plies; otherwise one element per ply (C0
    at interfaces), and with probability 1/2 (split_plies: always / never) one
    ply gets an extra thickness knot of random multiplicity inside it, so it
    holds two thickness elements (any through-thickness discretization)."""
    p1 = int(rng.integers(1, 4)) if p is None else p
    p2 = int(rng.integers(1, 4)) if p is None else p
    q = int(rng.integers(1, 5)) if q is None else q

    def knots(pp, ne):
        inner = np.sort(rng.uniform(0.05, 0.95, size=ne - 1))
        if ne >= 3 and pp >= 2:
            inner = np.sort(np.concatenate([inner, inner[:1]]))  # one C^{p-2} knot
        return np.concatenate([np.zeros(pp + 1), inner, np.ones(pp + 1)])

    k1 = knots(p1, int(rng.integers(1, 4)))
    k2 = knots(p2, int(rng.integers(1, 4)))
    m = int(rng.integers(1, max_ply + 1))
    iface = np.concatenate([[0.0], np.sort(rng.uniform(0.1, 0.9, size=m - 1)), [1.0]])
    if paper_regime:
        k3 = np.concatenate([np.zeros(q + 1), np.ones(q + 1)])
    else:
        k3 = layerwise_knots(q, iface)
    if sheared:
        J = np.array([[1.3, 0.2, 0.0], [-0.1, 0.9, 0.0], [0.05, -0.03, 0.15]])
    else:
        J = box_jac(1.0, 0.8, 0.1)
    if anisotropic:
        mats = [random_anisotropic(rng) for _ in range(n_mat)]
    else:
        mats = [material(jittered(CARBON, rng)) for _ in range(n_mat)]
    ply_mat = rng.integers(0, n_mat, size=m).astype(np.int32)
    theta = rng.uniform(0, np.pi, size=m)
    if not paper_regime:
        split = rng.uniform() < 0.5 if split_plies is None else split_plies
        l = int(rng.integers(0, m))
        t = iface[l] + (iface[l + 1] - iface[l]) * rng.uniform(0.25, 0.75)
        mult = int(rng.integers(1, q + 1))
        if split:
            k3 = np.sort(np.concatenate([k3, np.full(mult, t)]))
    return Laminate(p1=p1, k1=k1, p2=p2, k2=k2, q=q, k3=k3, jac=J, iface=iface, ply_mat=ply_mat,
                    theta=theta, C=np.stack(mats), name="random_small")


def greville(p: int, t: np.ndarray) -> np.ndarray:
    """Greville abscissae of an open knot vector (knot averages)."""
    n = len(t) - p - 1
    if p == 0:
        return 0.5 * (t[:n] + t[1:n + 1])
    return np.array([t[i + 1:i + p + 1].mean() for i in range(n)])


def control_points(lam: Laminate) -> np.ndarray:
    """Physical positions of the control points, in global function order
    (i1 fastest, then i2, then i_t), for the affine map x = DF xi."""
    g1, g2, g3 = greville(lam.p1, lam.k1), greville(lam.p2, lam.k2), greville(lam.q, lam.k3)
    T, Y, X = np.meshgrid(g3, g2, g1, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), T.ravel()], axis=1)
    return xi @ np.asarray(lam.jac).T
