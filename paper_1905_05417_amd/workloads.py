"""Seeded synthetic laminates (inputs only; no assembly arithmetic here).

Both the GPU path and the CPU oracle are fed from this module and nothing
else is shared between them.  A `Laminate` carries everything the operator
needs: open knot vectors (in-plane degrees p1, p2, thickness degree q), the
constant map gradient of the extruded box, the ply stack and the materials.

Workloads mirror the paper's setting (Sec. 4: flat plate, tensor-product
B-splines in-plane, plies stacked [0/90]... or [0/45/-45/90]..., orthotropic
plies rotated about the plate normal), at the sizes used by the tests and the
benchmark, and the shells of Sec. 2.3 (a curved B-spline or NURBS mid-surface
extruded along a constant vector) with materials varying in the plane
(Assumption 3).  Readings fixed here (the paper leaves them open):
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
    C: np.ndarray              # (n_mat,6,6) material axes; (n_mat, n1*n2, 6, 6) with mat_field
    ng: tuple = (0, 0, 0)
    name: str = ""
    meta: dict = field(default_factory=dict)
    # curved extruded shell F(xi) = S(xi1, xi2) + xi3 a_ext (jac unused when ctrl is set)
    ctrl: np.ndarray | None = None     # (n1*n2, 3) control points of S, in-plane function order
    weights: np.ndarray | None = None  # (n1*n2,) NURBS weights, or None for B-splines
    a_ext: np.ndarray | None = None    # (3,) extrusion vector
    mat_field: bool = False            # C varies in the plane: one 6x6 per material and in-plane function

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


# --------------------------------------------------------------- shells ----
def _blossom_coeffs(p: int, t: np.ndarray):
    """Per basis function i of degree p on knots t: (mean of t[i+1..i+p],
    mean of t_j t_k over pairs j < k of them), the B-spline coefficients of
    xi and xi^2 (their blossoms), so that sum_i c_i N_i reproduces them exactly."""
    n = len(t) - p - 1
    m1, m2 = np.zeros(n), np.zeros(n)
    for i in range(n):
        u = t[i + 1:i + p + 1]
        m1[i] = u.mean() if p > 0 else 0.5 * (t[i] + t[i + 1])
        if p >= 2:
            m2[i] = sum(u[j] * u[k] for j in range(p) for k in range(j + 1, p)) / (p * (p - 1) / 2)
    return m1, m2


def flat_shell(lam: Laminate) -> Laminate:
    """The same laminate described as a shell: S(xi1, xi2) = DF (xi1, xi2, 0)
    by control points at the Greville abscissae (B-splines reproduce linear
    maps), extruded along DF e3."""
    import copy
    out = copy.copy(lam)
    g1, g2 = greville(lam.p1, lam.k1), greville(lam.p2, lam.k2)
    Y, X = np.meshgrid(g2, g1, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    J = np.asarray(lam.jac, dtype=np.float64)
    out.ctrl = xi @ J.T
    out.a_ext = J[:, 2].copy()
    out.weights = None
    out.name = lam.name + "_as_shell"
    return out


def curved_shell(p, ne, q, angles_deg, mats, ply_mat, H=0.02, Lx=1.0, Ly=1.0, shear=0.3, bump=0.2, name="",
                 ne2=None, p2=None) -> Laminate:
    """A curved B-spline shell: S(xi) = (Lx xi1, Ly xi2 + shear xi1 (1 - xi1),
    bump (xi1 xi2 + xi1 (1 - xi1))) extruded along (0, 0, H), its control
    points the blossoms of these quadratics (exact for p >= 2).  Its map
    gradient varies over the plane while det DF = Lx Ly H (the projection on
    the xy-plane is a shear), so the shell's volume is Lx Ly H."""
    p2 = p if p2 is None else p2
    if min(p, p2) < 2:
        raise ValueError("curved_shell reproduces quadratics: degree >= 2")
    lam = plate(p, ne, q, angles_deg, mats, ply_mat, H=H, L=(Lx, Ly), name=name, ne2=ne2, p2=p2)
    a1, q1 = _blossom_coeffs(lam.p1, lam.k1)
    a2, _ = _blossom_coeffs(lam.p2, lam.k2)
    A2, A1 = np.meshgrid(a2, a1, indexing="ij")
    Q1 = np.meshgrid(a2, q1, indexing="ij")[1]
    x = Lx * A1
    y = Ly * A2 + shear * (A1 - Q1)
    z = bump * (A1 * A2 + (A1 - Q1))
    lam.ctrl = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    lam.a_ext = np.array([0.0, 0.0, H])
    lam.weights = None
    return lam


def _insert_knot(p, t, P, w, u):
    """Boehm's knot insertion in homogeneous coordinates: knot u once into the
    degree-p curve with knots t, control points P (n, d) and weights w (n,)."""
    n = len(t) - p - 1
    k = np.searchsorted(t, u, side="right") - 1
    Pw = np.concatenate([P * w[:, None], w[:, None]], axis=1)
    Q = np.zeros((n + 1, Pw.shape[1]))
    for i in range(n + 1):
        if i <= k - p:
            Q[i] = Pw[i]
        elif i > k:
            Q[i] = Pw[i - 1]
        else:
            a = (u - t[i]) / (t[i + p] - t[i])
            Q[i] = a * Pw[i] + (1 - a) * Pw[i - 1]
    t2 = np.insert(t, k + 1, u)
    return t2, Q[:, :-1] / Q[:, -1:], Q[:, -1].copy()


def nurbs_annulus_shell(ne1, ne2, q, angles_deg, mats, ply_mat, r0=0.6, r1=1.0, H=0.02, bump=0.15, name="",
                        p2=1) -> Laminate:
    """A quarter annulus (radii r0..r1, angle 0..pi/2) in the xy-plane as an
    exact NURBS surface, degree 2 around (the standard quarter circle: weights
    1, sqrt(2)/2, 1, refined by knot insertion) and degree p2 across, lifted
    by z = bump * x * y at the control points and extruded along (0, 0, H)."""
    p1 = 2
    t1 = np.array([0, 0, 0, 1, 1, 1], dtype=np.float64)
    arc = np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    w1 = np.array([1.0, np.sqrt(0.5), 1.0])
    for u in np.arange(1, ne1) / ne1:
        t1, arc, w1 = _insert_knot(p1, t1, arc, w1, u)
    k2 = open_uniform_knots(p2, ne2)
    radii = r0 + (r1 - r0) * greville(p2, k2)
    n1, n2 = len(w1), len(radii)
    ctrl = np.zeros((n2, n1, 3))
    for i2 in range(n2):
        ctrl[i2, :, 0] = radii[i2] * arc[:, 0]
        ctrl[i2, :, 1] = radii[i2] * arc[:, 1]
    ctrl[:, :, 2] = bump * ctrl[:, :, 0] * ctrl[:, :, 1]
    m = len(angles_deg)
    iface = uniform_iface(m)
    lam = Laminate(p1=p1, k1=t1, p2=p2, k2=k2, q=q, k3=layerwise_knots(q, iface), jac=box_jac(1.0, 1.0, H),
                   iface=iface, ply_mat=np.asarray(ply_mat, dtype=np.int32), theta=deg(angles_deg),
                   C=np.stack([np.asarray(c, dtype=np.float64) for c in mats]), name=name)
    lam.ctrl = ctrl.reshape(-1, 3)
    lam.weights = np.tile(w1, n2)
    lam.a_ext = np.array([0.0, 0.0, H])
    return lam


def linear_material_field(lam: Laminate, C1: np.ndarray) -> Laminate:
    """The laminate's materials varying linearly across the plane:
    C_m(xi) = C_m + xi1 C1[m], given per in-plane function by the coefficient
    at its Greville abscissa (B-splines reproduce linear functions)."""
    import copy
    out = copy.copy(lam)
    g1 = greville(lam.p1, lam.k1)
    gam = np.tile(g1, lam.n2)  # in-plane function order i1 + n1 * i2
    C0 = np.asarray(lam.C, dtype=np.float64)
    out.C = C0[:, None, :, :] + gam[None, :, None, None] * np.asarray(C1, dtype=np.float64)[:, None, :, :]
    out.mat_field = True
    out.name = lam.name + "_linear_field"
    return out


def smooth_material_field(lam: Laminate, rng: np.random.Generator, amp=0.3, sym=0.02) -> Laminate:
    """Seeded in-plane variation of every material: each in-plane function's
    6x6 is the material's scaled by 1 + amp * (a smooth random function of
    its Greville point), plus a seeded symmetric perturbation of entries up to
    a few times sym * max |C| (which can make a 6x6 indefinite: shear moduli
    are far below that).  sym = 0 keeps every control tensor a positive
    multiple of the material, so the field (a nonnegative partition of unity
    of them) and K stay positive definite."""
    import copy
    out = copy.copy(lam)
    g1, g2 = greville(lam.p1, lam.k1), greville(lam.p2, lam.k2)
    Y, X = np.meshgrid(g2, g1, indexing="ij")
    C0 = np.asarray(lam.C, dtype=np.float64)
    fields = []
    for m in range(C0.shape[0]):
        a, b, c = rng.uniform(0, 2 * np.pi, size=3)
        f = 1.0 + amp * np.sin(2 * X + a) * np.cos(3 * Y + b) + 0.5 * amp * np.sin(X + Y + c)
        E = rng.standard_normal((6, 6))
        E = sym * np.abs(C0[m]).max() * (E + E.T)
        fields.append(f.ravel()[:, None, None] * C0[m][None] + np.sin(5 * X + c).ravel()[:, None, None] * E[None])
    out.C = np.stack(fields)
    out.mat_field = True
    out.name = lam.name + "_field"
    return out


def shell_control_points(lam: Laminate) -> np.ndarray:
    """Control points of the map x = F(xi) in global function order (i1
    fastest, then i2, then i_t): ctrl_is + gamma_t a for a shell (B-splines in
    the thickness reproduce xi3 by its Greville abscissae); for an affine
    laminate, the control_points of DF xi."""
    if lam.ctrl is None:
        return control_points(lam)
    g3 = greville(lam.q, lam.k3)
    X = np.asarray(lam.ctrl, dtype=np.float64).reshape(-1, 3)
    a = np.asarray(lam.a_ext, dtype=np.float64)
    return (X[None, :, :] + g3[:, None, None] * a[None, None, :]).reshape(-1, 3)
