/*
 * oracle.c -- CPU reference for the layered 3D stiffness matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * GPU path.
 *
 * What it computes (Antolin, "Fast assembly of Galerkin matrices for 3D solid
 * laminated composites ...", arXiv 1905.05417):
 *
 *   K^{ij} = sum_l  int_{Omega_l} B^i(xi)^T D_l B^j(xi) |DF| dxi      (Sec. 2.3, eq. Km_0)
 *
 * by the standard method of Sec. 2.4: element by element, layer by layer,
 * tensor Gauss-Legendre quadrature on every (in-plane element x ply x
 * through-thickness knot span) cell.  Everything is FP64 and written for
 * obviousness, not speed:
 *   - basis functions: tensor products S(xi1,xi2) T(xi3) of B-splines
 *     (Assumption 1, Sec. 2.2), evaluated by the Cox-de Boor recursion;
 *   - strain-displacement matrix B (eq. B_0 / B_1) in Voigt order
 *     (11,22,33,12,13,23) with engineering shears.  The third column (u_3) is
 *     (0,0,d3,0,d1,d2): the printed equation repeats d3 in the last entry,
 *     which cannot be right because gamma_23 = du_2/dx_3 + du_3/dx_2;
 *   - physical gradients by the pull-back grad B = DF^{-T} grad_hat B (eq. gradient),
 *     either for a constant map gradient DF (an affine extrusion) or for the
 *     extrusion of a curved mid-surface, F(xi) = S(xi1, xi2) + xi3 a
 *     (Assumption 2, eq. extrusion), S given by control points on the
 *     in-plane basis, with DF = [dS/dxi1 | dS/dxi2 | a] evaluated at every
 *     Gauss point;
 *   - in-plane basis: B-splines, or NURBS (Sec. 2.2) when weights are given,
 *     R^i = w_i N^i / sum_k w_k N^k, used for the geometry and the
 *     displacement alike;
 *   - ply materials constant, or varying in the plane (Assumption 3): a
 *     6x6 per material and in-plane control function, C_m(xi) = sum_i R^i(xi) C_{m,i};
 *   - the ply tensor D_l: the 6x6 given in material axes is expanded to the
 *     fourth-order tensor, rotated by theta about +e3 with four rotation
 *     matrices, and folded back to Voigt form (eq. D).
 *
 * Also here, as plain definitions used to pin the paper's identities in tests:
 * the 2D operators P (eq. P), the 1D operators Q (eq. Q, with the test
 * function on the first factor), and the gradient of L = <G, K> with respect
 * to every ply's D_l, each material's 6x6 and every ply angle.
 *
 * Numbering (Assumption 1 and eq. a_0): in-plane function i_s = i1 + n1*i2,
 * global function i = i_t*n_s + i_s, degree of freedom 3*i + r.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t p1, p2, q;
  int32_t nk1, nk2, nk3;
  const double *k1, *k2, *k3;
  double J[9];            /* DF, row-major: J[a*3+b] = d x_a / d xi_b */
  int32_t n_ply;
  const double *iface;    /* n_ply+1 interfaces in [0,1], strictly increasing */
  const int32_t *ply_mat; /* material of every ply, bottom to top */
  const double *ply_theta;/* ply angle in radians, counterclockwise about +e3 */
  int32_t n_mat;
  const double *C;        /* n_mat 6x6 Voigt matrices in material axes, row-major
                             (n_mat * n1*n2 of them when mat_field is set) */
  int32_t ng1, ng2, ngz;  /* Gauss points per element direction / per z cell */
  /* Curved extruded shell (optional): when ctrl is not NULL, F(xi) = S(xi1,xi2) + xi3 a
   * with S(xi1,xi2) = sum_i R^i(xi1,xi2) ctrl_i, and J is not used. */
  const double *ctrl;     /* n1*n2 control points (x,y,z), in-plane function order i1 + n1*i2 */
  const double *wts;      /* NULL (B-splines) or n1*n2 positive weights (NURBS) */
  double a[3];            /* extrusion vector */
  int32_t mat_field;      /* 1: C holds a 6x6 per material and in-plane function */
} or_problem;

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1]: Newton iteration on the Legendre polynomial
 * P_n, evaluated with Bonnet's three-term recurrence. */
int or_gauss_legendre(int n, double *x, double *w) {
  if (n < 1 || n > 64) return -1;
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p0 = 1.0; p1 = z; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* B-splines (Cox-de Boor).  On the knot interval [t_s, t_{s+1}) of nonzero
 * length, the p+1 functions N_{s-p..s} are nonzero.  N[a], dN[a] receive
 * N_{s-p+a}(x) and its first derivative. */
static double safe_div(double a, double b) { return b != 0.0 ? a / b : 0.0; }

static void bspline_on_span(int p, const double *t, int s, double x, double *N, double *dN) {
  /* tab[k][a] = N_{s-k+a, k}(x), a = 0..k  (degree-k functions nonzero on span s) */
  double tab[16][16];
  tab[0][0] = 1.0;
  for (int k = 1; k <= p; ++k) {
    for (int a = 0; a <= k; ++a) {
      int i = s - k + a; /* function index N_{i,k} */
      double left = 0.0, right = 0.0;
      if (a >= 1) /* N_{i,k-1} is tab[k-1][a-1] */
        left = safe_div(x - t[i], t[i + k] - t[i]) * tab[k - 1][a - 1];
      if (a <= k - 1) /* N_{i+1,k-1} is tab[k-1][a] */
        right = safe_div(t[i + k + 1] - x, t[i + k + 1] - t[i + 1]) * tab[k - 1][a];
      tab[k][a] = left + right;
    }
  }
  for (int a = 0; a <= p; ++a) N[a] = tab[p][a];
  for (int a = 0; a <= p; ++a) {
    if (p == 0) { dN[a] = 0.0; continue; }
    int i = s - p + a;
    double d = 0.0;
    if (a >= 1) d += safe_div((double)p, t[i + p] - t[i]) * tab[p - 1][a - 1];
    if (a <= p - 1) d -= safe_div((double)p, t[i + p + 1] - t[i + 1]) * tab[p - 1][a];
    dN[a] = d;
  }
}

static int n_funcs(int p, int nk) { return nk - p - 1; }

/* Knot interval containing x; at the right end, the last interval of nonzero length. */
static int find_span(int p, int nk, const double *t, double x) {
  int n = n_funcs(p, nk);
  if (x >= t[n]) {
    int s = n - 1;
    while (s > p && !(t[s + 1] > t[s])) --s;
    return s;
  }
  int s = p;
  while (s < n - 1 && !(x < t[s + 1])) ++s;
  return s;
}

/* Every basis function (all n of them) and its derivative at x. */
int or_bspline_eval(int p, int nk, const double *t, double x, double *N_all, double *dN_all) {
  if (p < 0 || p > 15 || nk < 2 * p + 2) return -1;
  int n = n_funcs(p, nk);
  for (int i = 0; i < n; ++i) N_all[i] = dN_all[i] = 0.0;
  int s = find_span(p, nk, t, x);
  double N[16], dN[16];
  bspline_on_span(p, t, s, x, N, dN);
  for (int a = 0; a <= p; ++a) {
    N_all[s - p + a] = N[a];
    dN_all[s - p + a] = dN[a];
  }
  return 0;
}

/* Intervals of nonzero length: their knot indices, in increasing order. */
static int nonzero_spans(int p, int nk, const double *t, int *spans) {
  int n = n_funcs(p, nk), c = 0;
  for (int s = p; s <= n - 1; ++s)
    if (t[s + 1] > t[s]) spans[c++] = s;
  return c;
}

/* 1D support overlap: adj[i*(2p+1) + c] lists (sorted) the j whose support
 * shares an interval of nonzero length with that of i; cnt[i] is their number. */
static void overlap_1d(int p, int nk, const double *t, int *cnt, int *adj) {
  int n = n_funcs(p, nk);
  int w = 2 * p + 1;
  int *mark = (int *)calloc((size_t)n, sizeof(int));
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) mark[j] = 0;
    for (int s = i; s <= i + p && s <= n - 1; ++s) {
      if (s < p || !(t[s + 1] > t[s])) continue;
      for (int j = s - p; j <= s; ++j) mark[j] = 1;
    }
    int c = 0;
    for (int j = 0; j < n; ++j)
      if (mark[j]) adj[i * w + c++] = j;
    cnt[i] = c;
  }
  free(mark);
}

/* ------------------------------------------------------------------------ */
/* Elasticity tensor in Voigt form and its rotation about +e3 (eq. D). */
static const int VI[6] = {0, 1, 2, 0, 0, 1};
static const int VJ[6] = {0, 1, 2, 1, 2, 2};
static int voigt_of(int i, int j) {
  if (i == j) return i;
  int a = i < j ? i : j, b = i < j ? j : i;
  if (a == 0 && b == 1) return 3;
  if (a == 0 && b == 2) return 4;
  return 5;
}

static void tensor_from_voigt(const double *D, double T[3][3][3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) T[i][j][k][l] = D[voigt_of(i, j) * 6 + voigt_of(k, l)];
}

static void voigt_from_tensor(double T[3][3][3][3], double *D) {
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) D[I * 6 + J] = T[VI[I]][VJ[I]][VI[J]][VJ[J]];
}

/* R[i][p] = e_i . a_p, with material axes a_1 = (c, s, 0), a_2 = (-s, c, 0), a_3 = e_3. */
static void rot_matrix(double th, double R[3][3], double dR[3][3]) {
  double c = cos(th), s = sin(th);
  double r[3][3] = {{c, -s, 0.0}, {s, c, 0.0}, {0.0, 0.0, 1.0}};
  double d[3][3] = {{-s, -c, 0.0}, {c, -s, 0.0}, {0.0, 0.0, 0.0}};
  memcpy(R, r, sizeof r);
  memcpy(dR, d, sizeof d);
}

/* C'_{ijkl} = A_ip B_jq E_kr F_ls C_pqrs */
static void rotate4(double A[3][3], double B[3][3], double E[3][3], double F[3][3],
                    double T[3][3][3][3], double out[3][3][3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double acc = 0.0;
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q)
              for (int r = 0; r < 3; ++r)
                for (int s = 0; s < 3; ++s) acc += A[i][p] * B[j][q] * E[k][r] * F[l][s] * T[p][q][r][s];
          out[i][j][k][l] = acc;
        }
}

/* D(theta) for a 6x6 given in material axes. */
int or_rotate_voigt(const double *C6, double theta, double *D6) {
  double T[3][3][3][3], U[3][3][3][3], R[3][3], dR[3][3];
  tensor_from_voigt(C6, T);
  rot_matrix(theta, R, dR);
  rotate4(R, R, R, R, T, U);
  voigt_from_tensor(U, D6);
  return 0;
}

/* dD/dtheta: product rule over the four rotation factors. */
int or_rotate_voigt_dtheta(const double *C6, double theta, double *dD6) {
  double T[3][3][3][3], U[3][3][3][3], R[3][3], dR[3][3];
  double acc[36];
  tensor_from_voigt(C6, T);
  rot_matrix(theta, R, dR);
  for (int a = 0; a < 36; ++a) acc[a] = 0.0;
  for (int f = 0; f < 4; ++f) {
    rotate4(f == 0 ? dR : R, f == 1 ? dR : R, f == 2 ? dR : R, f == 3 ? dR : R, T, U);
    double tmp[36];
    voigt_from_tensor(U, tmp);
    for (int a = 0; a < 36; ++a) acc[a] += tmp[a];
  }
  memcpy(dD6, acc, sizeof acc);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Strain-displacement matrix for one scalar basis function with physical
 * gradient g: column r is the Voigt strain of the displacement e_r * B. */
static void bmat(const double g[3], double B[6][3]) {
  memset(B, 0, sizeof(double) * 18);
  B[0][0] = g[0];
  B[1][1] = g[1];
  B[2][2] = g[2];
  B[3][0] = g[1]; B[3][1] = g[0];
  B[4][0] = g[2]; B[4][2] = g[0];
  B[5][1] = g[2]; B[5][2] = g[1];
}

/* out(3x3) = Ba^T D Bb */
static void btdb(double Ba[6][3], const double *D, double Bb[6][3], double out[3][3]) {
  double DB[6][3];
  for (int I = 0; I < 6; ++I)
    for (int s = 0; s < 3; ++s) {
      double acc = 0.0;
      for (int J = 0; J < 6; ++J) acc += D[I * 6 + J] * Bb[J][s];
      DB[I][s] = acc;
    }
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s) {
      double acc = 0.0;
      for (int I = 0; I < 6; ++I) acc += Ba[I][r] * DB[I][s];
      out[r][s] = acc;
    }
}

static int inv3(const double *J, double *Ji, double *det) {
  double a = J[0], b = J[1], c = J[2], d = J[3], e = J[4], f = J[5], g = J[6], h = J[7], k = J[8];
  double A = e * k - f * h, B = -(d * k - f * g), Cc = d * h - e * g;
  double dt = a * A + b * B + c * Cc;
  if (!(fabs(dt) > 0.0) || !isfinite(dt)) return -1;
  Ji[0] = A / dt; Ji[1] = -(b * k - c * h) / dt; Ji[2] = (b * f - c * e) / dt;
  Ji[3] = B / dt; Ji[4] = (a * k - c * g) / dt;  Ji[5] = -(a * f - c * d) / dt;
  Ji[6] = Cc / dt; Ji[7] = -(a * h - b * g) / dt; Ji[8] = (a * e - b * d) / dt;
  *det = dt;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Problem bookkeeping. */
typedef struct {
  or_problem P;
  int n1, n2, nt, ns;
  int ns1, ns2, ns3;        /* number of nonzero knot intervals per direction */
  int *sp1, *sp2, *sp3;     /* their knot indices */
  int w1, w2, w3;           /* 2p+1 widths of the overlap lists */
  int *c1, *a1, *c2, *a2, *c3, *a3;
  double Ji[9], detJ;
  double *Dply;             /* n_ply*36, rotated ply tensors */
  double *gx1, *gw1, *gx2, *gw2, *gx3, *gw3;
} ctx;

static void ctx_free(ctx *c) {
  free(c->sp1); free(c->sp2); free(c->sp3);
  free(c->c1); free(c->a1); free(c->c2); free(c->a2); free(c->c3); free(c->a3);
  free(c->Dply);
  free(c->gx1); free(c->gw1); free(c->gx2); free(c->gw2); free(c->gx3); free(c->gw3);
}

/* In-plane parametric point of Gauss point (g1, g2) of the element with knot
 * intervals s1, s2, and the element's half lengths. */
static void point_coords(const ctx *c, int s1, int s2, int g1, int g2, double *x1, double *x2, double *h1,
                         double *h2) {
  const or_problem *P = &c->P;
  double a1 = P->k1[s1], b1 = P->k1[s1 + 1], a2 = P->k2[s2], b2 = P->k2[s2 + 1];
  *h1 = 0.5 * (b1 - a1);
  *h2 = 0.5 * (b2 - a2);
  *x1 = 0.5 * (a1 + b1) + *h1 * c->gx1[g1];
  *x2 = 0.5 * (a2 + b2) + *h2 * c->gx2[g2];
}

/* The (p1+1)(p2+1) in-plane functions nonzero on element (s1, s2) at (x1, x2):
 * values R and derivatives dR1 = dR/dxi1, dR2 = dR/dxi2, local index
 * b = b2*(p1+1) + b1 for the function (s1-p1+b1, s2-p2+b2).  B-spline
 * products; with weights, the NURBS quotient R = w N / W, W = sum w N, and
 * its derivative by the quotient rule. */
static void inplane_basis(const ctx *c, int s1, int s2, double x1, double x2, double *R, double *dR1,
                          double *dR2) {
  const or_problem *P = &c->P;
  int p1 = P->p1, p2 = P->p2;
  double N1[16], d1[16], N2[16], d2[16];
  bspline_on_span(p1, P->k1, s1, x1, N1, d1);
  bspline_on_span(p2, P->k2, s2, x2, N2, d2);
  for (int b2 = 0; b2 <= p2; ++b2)
    for (int b1 = 0; b1 <= p1; ++b1) {
      int b = b2 * (p1 + 1) + b1;
      R[b] = N1[b1] * N2[b2];
      dR1[b] = d1[b1] * N2[b2];
      dR2[b] = N1[b1] * d2[b2];
    }
  if (!P->wts) return;
  int nb = (p1 + 1) * (p2 + 1);
  double W = 0.0, W1 = 0.0, W2 = 0.0, w[256];
  for (int b2 = 0; b2 <= p2; ++b2)
    for (int b1 = 0; b1 <= p1; ++b1) {
      int b = b2 * (p1 + 1) + b1;
      w[b] = P->wts[(s2 - p2 + b2) * c->n1 + (s1 - p1 + b1)];
      W += w[b] * R[b];
      W1 += w[b] * dR1[b];
      W2 += w[b] * dR2[b];
    }
  for (int b = 0; b < nb; ++b) {
    double r = w[b] * R[b] / W;
    dR1[b] = (w[b] * dR1[b] - r * W1) / W;
    dR2[b] = (w[b] * dR2[b] - r * W2) / W;
    R[b] = r;
  }
}

/* DF^{-1} (row-major) and det DF at an in-plane point of element (s1, s2):
 * the constant map, or DF = [dS/dxi1 | dS/dxi2 | a] for the curved
 * extrusion, dS/dxi_k = sum_b dR_k[b] ctrl(b).  Returns -1 if singular. */
static int point_geometry(const ctx *c, int s1, int s2, const double *dR1, const double *dR2, double *Ji,
                          double *det) {
  const or_problem *P = &c->P;
  if (!P->ctrl) {
    memcpy(Ji, c->Ji, sizeof(double) * 9);
    *det = c->detJ;
    return 0;
  }
  int p1 = P->p1, p2 = P->p2;
  double S1[3] = {0, 0, 0}, S2[3] = {0, 0, 0};
  for (int b2 = 0; b2 <= p2; ++b2)
    for (int b1 = 0; b1 <= p1; ++b1) {
      int b = b2 * (p1 + 1) + b1;
      const double *X = P->ctrl + 3 * (size_t)((s2 - p2 + b2) * c->n1 + (s1 - p1 + b1));
      for (int k = 0; k < 3; ++k) {
        S1[k] += dR1[b] * X[k];
        S2[k] += dR2[b] * X[k];
      }
    }
  double J[9];
  for (int k = 0; k < 3; ++k) {
    J[3 * k + 0] = S1[k];
    J[3 * k + 1] = S2[k];
    J[3 * k + 2] = P->a[k];
  }
  return inv3(J, Ji, det);
}

/* The rotated tensor of ply l at an in-plane point with basis values R on
 * element (s1, s2): the constant one, or the rotation of
 * C_m(xi) = sum_b R[b] C_{m, function b} for a material field. */
static void point_material(const ctx *c, int l, int s1, int s2, const double *R, double *D) {
  const or_problem *P = &c->P;
  if (!P->mat_field) {
    memcpy(D, c->Dply + 36 * (size_t)l, sizeof(double) * 36);
    return;
  }
  int p1 = P->p1, p2 = P->p2;
  double Cx[36] = {0};
  for (int b2 = 0; b2 <= p2; ++b2)
    for (int b1 = 0; b1 <= p1; ++b1) {
      int b = b2 * (p1 + 1) + b1;
      size_t is = (size_t)(s2 - p2 + b2) * c->n1 + (s1 - p1 + b1);
      const double *Cc = P->C + 36 * ((size_t)P->ply_mat[l] * c->ns + is);
      for (int e = 0; e < 36; ++e) Cx[e] += R[b] * Cc[e];
    }
  or_rotate_voigt(Cx, P->ply_theta[l], D);
}

/* Open knot vector on [0,1]: p+1 zeros, non-decreasing interior, p+1 ones. */
static int check_knots(int p, int nk, const double *t) {
  if (p < 0 || p > 15 || nk < 2 * p + 2) return -1;
  for (int i = 0; i < nk; ++i)
    if (!isfinite(t[i])) return -1;
  for (int i = 0; i + 1 < nk; ++i)
    if (!(t[i + 1] >= t[i])) return -1;
  for (int i = 0; i <= p; ++i)
    if (t[i] != 0.0 || t[nk - 1 - i] != 1.0) return -1;
  return 0;
}

static int ctx_init(ctx *c, const or_problem *P) {
  memset(c, 0, sizeof *c);
  c->P = *P;
  if (check_knots(P->p1, P->nk1, P->k1) || check_knots(P->p2, P->nk2, P->k2) ||
      check_knots(P->q, P->nk3, P->k3))
    return -1;
  if (P->n_ply < 1 || P->n_mat < 1) return -1;
  if (P->iface[0] != P->k3[0] || P->iface[P->n_ply] != P->k3[P->nk3 - 1]) return -1;
  for (int l = 0; l < P->n_ply; ++l) {
    if (!(P->iface[l + 1] > P->iface[l])) return -1;
    if (P->ply_mat[l] < 0 || P->ply_mat[l] >= P->n_mat) return -1;
  }
  if (!P->ctrl && inv3(P->J, c->Ji, &c->detJ)) return -1;
  c->n1 = n_funcs(P->p1, P->nk1);
  c->n2 = n_funcs(P->p2, P->nk2);
  c->nt = n_funcs(P->q, P->nk3);
  c->ns = c->n1 * c->n2;
  if (P->ctrl) {
    for (int e = 0; e < 3 * c->ns; ++e)
      if (!isfinite(P->ctrl[e])) return -1;
    for (int e = 0; e < 3; ++e)
      if (!isfinite(P->a[e])) return -1;
  }
  if (P->wts)
    for (int e = 0; e < c->ns; ++e)
      if (!(P->wts[e] > 0.0) || !isfinite(P->wts[e])) return -1;
  c->sp1 = (int *)malloc(sizeof(int) * (size_t)P->nk1);
  c->sp2 = (int *)malloc(sizeof(int) * (size_t)P->nk2);
  c->sp3 = (int *)malloc(sizeof(int) * (size_t)P->nk3);
  c->ns1 = nonzero_spans(P->p1, P->nk1, P->k1, c->sp1);
  c->ns2 = nonzero_spans(P->p2, P->nk2, P->k2, c->sp2);
  c->ns3 = nonzero_spans(P->q, P->nk3, P->k3, c->sp3);
  c->w1 = 2 * P->p1 + 1; c->w2 = 2 * P->p2 + 1; c->w3 = 2 * P->q + 1;
  c->c1 = (int *)malloc(sizeof(int) * (size_t)c->n1);
  c->a1 = (int *)malloc(sizeof(int) * (size_t)c->n1 * c->w1);
  c->c2 = (int *)malloc(sizeof(int) * (size_t)c->n2);
  c->a2 = (int *)malloc(sizeof(int) * (size_t)c->n2 * c->w2);
  c->c3 = (int *)malloc(sizeof(int) * (size_t)c->nt);
  c->a3 = (int *)malloc(sizeof(int) * (size_t)c->nt * c->w3);
  overlap_1d(P->p1, P->nk1, P->k1, c->c1, c->a1);
  overlap_1d(P->p2, P->nk2, P->k2, c->c2, c->a2);
  overlap_1d(P->q, P->nk3, P->k3, c->c3, c->a3);
  c->Dply = (double *)malloc(sizeof(double) * 36 * (size_t)P->n_ply);
  const size_t per_mat = P->mat_field ? (size_t)c->ns : 1;
  for (size_t e = 0; e < 36 * per_mat * (size_t)P->n_mat; ++e)
    if (!isfinite(P->C[e])) return -1;
  for (int l = 0; l < P->n_ply; ++l)  /* constant materials: each ply's rotated tensor */
    or_rotate_voigt(P->C + 36 * per_mat * (size_t)P->ply_mat[l], P->ply_theta[l], c->Dply + 36 * (size_t)l);
  int g1 = P->ng1 > 0 ? P->ng1 : P->p1 + 1;
  int g2 = P->ng2 > 0 ? P->ng2 : P->p2 + 1;
  int g3 = P->ngz > 0 ? P->ngz : P->q + 1;
  c->P.ng1 = g1; c->P.ng2 = g2; c->P.ngz = g3;
  c->gx1 = (double *)malloc(sizeof(double) * g1); c->gw1 = (double *)malloc(sizeof(double) * g1);
  c->gx2 = (double *)malloc(sizeof(double) * g2); c->gw2 = (double *)malloc(sizeof(double) * g2);
  c->gx3 = (double *)malloc(sizeof(double) * g3); c->gw3 = (double *)malloc(sizeof(double) * g3);
  if (or_gauss_legendre(g1, c->gx1, c->gw1) || or_gauss_legendre(g2, c->gx2, c->gw2) ||
      or_gauss_legendre(g3, c->gx3, c->gw3))
    return -1;
  if (P->ctrl) /* a curved map must be invertible at every in-plane Gauss point */
    for (int z2 = 0; z2 < c->ns2; ++z2)
      for (int z1 = 0; z1 < c->ns1; ++z1)
        for (int b = 0; b < g2; ++b)
          for (int a = 0; a < g1; ++a) {
            double R[256], dR1[256], dR2[256], Ji[9], det, x1, x2, h1, h2;
            point_coords(c, c->sp1[z1], c->sp2[z2], a, b, &x1, &x2, &h1, &h2);
            inplane_basis(c, c->sp1[z1], c->sp2[z2], x1, x2, R, dR1, dR2);
            if (point_geometry(c, c->sp1[z1], c->sp2[z2], dR1, dR2, Ji, &det)) return -1;
          }
  return 0;
}

/* CSR of the full matrix: rows 3*i+r; columns (j_t, j2, j1, s) ascending. */
static int64_t row_len(const ctx *c, int it, int i2, int i1) {
  return (int64_t)3 * c->c3[it] * c->c2[i2] * c->c1[i1];
}

static void row_decode(const ctx *c, int64_t row, int *it, int *i2, int *i1, int *r) {
  int64_t i = row / 3;
  *r = (int)(row % 3);
  *it = (int)(i / c->ns);
  int is = (int)(i % c->ns);
  *i2 = is / c->n1;
  *i1 = is % c->n1;
}

static void row_columns(const ctx *c, int it, int i2, int i1, int32_t *col) {
  int64_t k = 0;
  for (int a = 0; a < c->c3[it]; ++a) {
    int jt = c->a3[it * c->w3 + a];
    for (int b = 0; b < c->c2[i2]; ++b) {
      int j2 = c->a2[i2 * c->w2 + b];
      for (int e = 0; e < c->c1[i1]; ++e) {
        int j1 = c->a1[i1 * c->w1 + e];
        int64_t j = (int64_t)jt * c->ns + (int64_t)j2 * c->n1 + j1;
        for (int s = 0; s < 3; ++s) col[k++] = (int32_t)(3 * j + s);
      }
    }
  }
}

int64_t or_pattern_size(const or_problem *P, int64_t *n_rows) {
  ctx c;
  if (ctx_init(&c, P)) { ctx_free(&c); return -1; }
  int64_t nnz = 0;
  for (int it = 0; it < c.nt; ++it)
    for (int i2 = 0; i2 < c.n2; ++i2)
      for (int i1 = 0; i1 < c.n1; ++i1) nnz += 3 * row_len(&c, it, i2, i1);
  if (n_rows) *n_rows = (int64_t)3 * c.ns * c.nt;
  ctx_free(&c);
  return nnz;
}

int or_pattern(const or_problem *P, int64_t *rowptr, int32_t *colind) {
  ctx c;
  if (ctx_init(&c, P)) { ctx_free(&c); return -1; }
  int64_t nrows = (int64_t)3 * c.ns * c.nt;
  rowptr[0] = 0;
  for (int64_t row = 0; row < nrows; ++row) {
    int it, i2, i1, r;
    row_decode(&c, row, &it, &i2, &i1, &r);
    rowptr[row + 1] = rowptr[row] + row_len(&c, it, i2, i1);
  }
  for (int64_t row = 0; row < nrows; ++row) {
    int it, i2, i1, r;
    row_decode(&c, row, &it, &i2, &i1, &r);
    row_columns(&c, it, i2, i1, colind + rowptr[row]);
  }
  ctx_free(&c);
  return 0;
}

static int64_t find_col(const int32_t *col, int64_t lo, int64_t hi, int32_t key) {
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

/* One quadrature cell: in-plane element (knot intervals s1, s2) times the
 * thickness interval [za, zb] inside knot interval s3.  The caller loops over
 * the cell's Gauss points; cell_point fills, for point (g1,g2,g3), the weight
 * and the physical gradients of the nloc = (p1+1)(p2+1)(q+1) local functions,
 * local index a = (at*(p2+1) + a2)*(p1+1) + a1, and (R) the values of the
 * (p1+1)(p2+1) in-plane functions. */
typedef struct {
  int s1, s2, s3;
  double za, zb;
} cell_t;

static double cell_point(const ctx *c, const cell_t *cl, int g1, int g2, int g3, double (*grad)[3], double *R) {
  const or_problem *P = &c->P;
  int p1 = P->p1, p2 = P->p2, q = P->q;
  double x1, x2, h1, h2;
  point_coords(c, cl->s1, cl->s2, g1, g2, &x1, &x2, &h1, &h2);
  double h3 = 0.5 * (cl->zb - cl->za);
  double x3 = 0.5 * (cl->za + cl->zb) + h3 * c->gx3[g3];
  double dR1[256], dR2[256], T[16], dT[16], Ji[9], det;
  inplane_basis(c, cl->s1, cl->s2, x1, x2, R, dR1, dR2);
  bspline_on_span(q, P->k3, cl->s3, x3, T, dT);
  if (point_geometry(c, cl->s1, cl->s2, dR1, dR2, Ji, &det)) return NAN;  /* excluded by ctx_init */
  int a = 0;
  for (int at = 0; at <= q; ++at)
    for (int b2 = 0; b2 <= p2; ++b2)
      for (int b1 = 0; b1 <= p1; ++b1, ++a) {
        int b = b2 * (p1 + 1) + b1;
        double gh[3] = {dR1[b] * T[at], dR2[b] * T[at], R[b] * dT[at]};
        /* grad = DF^{-T} gh:  grad_k = sum_m Ji[m][k] gh[m] */
        for (int k = 0; k < 3; ++k)
          grad[a][k] = Ji[0 * 3 + k] * gh[0] + Ji[1 * 3 + k] * gh[1] + Ji[2 * 3 + k] * gh[2];
      }
  return c->gw1[g1] * c->gw2[g2] * c->gw3[g3] * h1 * h2 * h3 * fabs(det);
}

static int64_t local_to_global(const ctx *c, const cell_t *cl, int a) {
  int p1 = c->P.p1, p2 = c->P.p2;
  int b1 = a % (p1 + 1);
  int b2 = (a / (p1 + 1)) % (p2 + 1);
  int at = a / ((p1 + 1) * (p2 + 1));
  int i1 = cl->s1 - p1 + b1, i2 = cl->s2 - p2 + b2, it = cl->s3 - c->P.q + at;
  return (int64_t)it * c->ns + (int64_t)i2 * c->n1 + i1;
}

/* Cells of one in-plane element column: every (ply, z interval) pair of
 * positive length.  Returns the count; cells (if not NULL) receive them in
 * bottom-to-top order, with the ply index in plies[]. */
static int column_cells(const ctx *c, int s1, int s2, cell_t *cells, int *plies) {
  int n = 0;
  for (int l = 0; l < c->P.n_ply; ++l)
    for (int z = 0; z < c->ns3; ++z) {
      int s3 = c->sp3[z];
      double za = fmax(c->P.iface[l], c->P.k3[s3]);
      double zb = fmin(c->P.iface[l + 1], c->P.k3[s3 + 1]);
      if (zb > za) {
        if (cells) {
          cells[n].s1 = s1; cells[n].s2 = s2; cells[n].s3 = s3;
          cells[n].za = za; cells[n].zb = zb;
          plies[n] = l;
        }
        ++n;
      }
    }
  return n;
}

/* Standard assembly (Sec. 2.4): for every in-plane element, every ply, every
 * z cell in the ply, accumulate the element matrix over the tensor Gauss rule
 * and add it into the CSR.  In-plane element stripes of one colour
 * (xi2 knot interval index mod p2+1) touch disjoint rows, so they run in
 * parallel without races and with a fixed summation order. */
int or_assemble(const or_problem *P, const int64_t *rowptr, const int32_t *colind, double *vals, int nthreads) {
  ctx c;
  if (ctx_init(&c, P)) { ctx_free(&c); return -1; }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int64_t nnz = rowptr[(int64_t)3 * c.ns * c.nt];
  for (int64_t e = 0; e < nnz; ++e) vals[e] = 0.0;
  const int nloc = (P->p1 + 1) * (P->p2 + 1) * (P->q + 1);
  const int ncell_max = column_cells(&c, c.sp1[0], c.sp2[0], NULL, NULL);
  for (int colour = 0; colour <= P->p2; ++colour) {
#pragma omp parallel
    {
      double (*grad)[3] = (double (*)[3])malloc(sizeof(double) * 3 * nloc);
      double (*Bm)[6][3] = (double (*)[6][3])malloc(sizeof(double) * 18 * nloc);
      double *Ke = (double *)malloc(sizeof(double) * 9 * (size_t)nloc * nloc);
      int64_t *glob = (int64_t *)malloc(sizeof(int64_t) * nloc);
      cell_t *cells = (cell_t *)malloc(sizeof(cell_t) * (size_t)(ncell_max > 0 ? ncell_max : 1));
      int *plies = (int *)malloc(sizeof(int) * (size_t)(ncell_max > 0 ? ncell_max : 1));
#pragma omp for schedule(dynamic, 1)
      for (int z2 = 0; z2 < c.ns2; ++z2) {
        int s2 = c.sp2[z2];
        if (s2 % (P->p2 + 1) != colour) continue;
        for (int z1 = 0; z1 < c.ns1; ++z1) {
          int s1 = c.sp1[z1];
          int ncell = column_cells(&c, s1, s2, cells, plies);
          for (int ic = 0; ic < ncell; ++ic) {
            const cell_t *cl = &cells[ic];
            memset(Ke, 0, sizeof(double) * 9 * (size_t)nloc * nloc);
            for (int g3 = 0; g3 < c.P.ngz; ++g3)
              for (int g2 = 0; g2 < c.P.ng2; ++g2)
                for (int g1 = 0; g1 < c.P.ng1; ++g1) {
                  double R[256], D[36];
                  double w = cell_point(&c, cl, g1, g2, g3, grad, R);
                  point_material(&c, plies[ic], cl->s1, cl->s2, R, D);
                  for (int a = 0; a < nloc; ++a) bmat(grad[a], Bm[a]);
                  for (int a = 0; a < nloc; ++a)
                    for (int b = 0; b < nloc; ++b) {
                      double blk[3][3];
                      btdb(Bm[a], D, Bm[b], blk);
                      for (int r = 0; r < 3; ++r)
                        for (int s = 0; s < 3; ++s)
                          Ke[((size_t)(3 * a + r)) * 3 * nloc + 3 * b + s] += w * blk[r][s];
                    }
                }
            for (int a = 0; a < nloc; ++a) glob[a] = local_to_global(&c, cl, a);
            for (int a = 0; a < nloc; ++a)
              for (int r = 0; r < 3; ++r) {
                int64_t row = 3 * glob[a] + r;
                int64_t lo = rowptr[row], hi = rowptr[row + 1];
                for (int b = 0; b < nloc; ++b)
                  for (int s = 0; s < 3; ++s) {
                    int32_t col = (int32_t)(3 * glob[b] + s);
                    int64_t pos = find_col(colind, lo, hi, col);
                    vals[pos] += Ke[((size_t)(3 * a + r)) * 3 * nloc + 3 * b + s];
                  }
              }
          }
        }
      }
      free(grad); free(Bm); free(Ke); free(glob); free(cells); free(plies);
    }
  }
  ctx_free(&c);
  return 0;
}

/* Selected rows only: row lengths (sel_col == NULL) or the rows themselves.
 * sel_ptr has nsel+1 entries (prefix sums of the lengths, filled by the
 * length call).  Each row is summed point by point over the cells of its test
 * function's support, so its last bits may differ from or_assemble, which
 * sums each cell's element matrix first. */
int or_assemble_rows(const or_problem *P, int64_t nsel, const int64_t *rows, int64_t *sel_ptr,
                     int32_t *sel_col, double *sel_vals, int nthreads) {
  ctx c;
  if (ctx_init(&c, P)) { ctx_free(&c); return -1; }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int64_t nrows = (int64_t)3 * c.ns * c.nt;
  for (int64_t k = 0; k < nsel; ++k)
    if (rows[k] < 0 || rows[k] >= nrows) { ctx_free(&c); return -1; }
  if (sel_col == NULL) {
    sel_ptr[0] = 0;
    for (int64_t k = 0; k < nsel; ++k) {
      int it, i2, i1, r;
      row_decode(&c, rows[k], &it, &i2, &i1, &r);
      sel_ptr[k + 1] = sel_ptr[k] + row_len(&c, it, i2, i1);
    }
    ctx_free(&c);
    return 0;
  }
  const int nloc = (P->p1 + 1) * (P->p2 + 1) * (P->q + 1);
  const int ncell_max = column_cells(&c, c.sp1[0], c.sp2[0], NULL, NULL);
#pragma omp parallel
  {
    double (*grad)[3] = (double (*)[3])malloc(sizeof(double) * 3 * nloc);
    double (*Bm)[6][3] = (double (*)[6][3])malloc(sizeof(double) * 18 * nloc);
    cell_t *cells = (cell_t *)malloc(sizeof(cell_t) * (size_t)(ncell_max > 0 ? ncell_max : 1));
    int *plies = (int *)malloc(sizeof(int) * (size_t)(ncell_max > 0 ? ncell_max : 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < nsel; ++k) {
      int it, i2, i1, r;
      row_decode(&c, rows[k], &it, &i2, &i1, &r);
      int64_t lo = sel_ptr[k], hi = sel_ptr[k + 1];
      row_columns(&c, it, i2, i1, sel_col + lo);
      for (int64_t e = lo; e < hi; ++e) sel_vals[e] = 0.0;
      int64_t gi = (int64_t)it * c.ns + (int64_t)i2 * c.n1 + i1;
      for (int z2 = 0; z2 < c.ns2; ++z2) {
        int s2 = c.sp2[z2];
        if (s2 < i2 || s2 > i2 + P->p2) continue;
        for (int z1 = 0; z1 < c.ns1; ++z1) {
          int s1 = c.sp1[z1];
          if (s1 < i1 || s1 > i1 + P->p1) continue;
          int ncell = column_cells(&c, s1, s2, cells, plies);
          for (int ic = 0; ic < ncell; ++ic) {
            const cell_t *cl = &cells[ic];
            if (cl->s3 < it || cl->s3 > it + P->q) continue;
            int aloc = -1;
            for (int a = 0; a < nloc; ++a)
              if (local_to_global(&c, cl, a) == gi) aloc = a;
            for (int g3 = 0; g3 < c.P.ngz; ++g3)
              for (int g2 = 0; g2 < c.P.ng2; ++g2)
                for (int g1 = 0; g1 < c.P.ng1; ++g1) {
                  double R[256], D[36];
                  double w = cell_point(&c, cl, g1, g2, g3, grad, R);
                  point_material(&c, plies[ic], cl->s1, cl->s2, R, D);
                  for (int a = 0; a < nloc; ++a) bmat(grad[a], Bm[a]);
                  for (int b = 0; b < nloc; ++b) {
                    double blk[3][3];
                    btdb(Bm[aloc], D, Bm[b], blk);
                    int64_t gj = local_to_global(&c, cl, b);
                    for (int s = 0; s < 3; ++s) {
                      int64_t pos = find_col(sel_col, lo, hi, (int32_t)(3 * gj + s));
                      sel_vals[pos] += w * blk[r][s];
                    }
                  }
                }
          }
        }
      }
    }
    free(grad); free(Bm); free(cells); free(plies);
  }
  ctx_free(&c);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Gradient of L = sum G .* K with respect to each ply's D_l:
 *   dL/dD_l[I][J] = sum_{cells in l} sum_g w sum_{a,b,r,s} G[(a,r),(b,s)] B_a[I][r] B_b[J][s]
 * (K is linear in D_l, eq. Km_0).  Per-stripe partial sums are reduced in a
 * fixed order. */
int or_grad_D(const or_problem *P, const int64_t *rowptr, const int32_t *colind, const double *G,
              double *dLdD, int nthreads) {
  ctx c;
  if (P->mat_field || ctx_init(&c, P)) { if (!P->mat_field) ctx_free(&c); return -1; }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const int nloc = (P->p1 + 1) * (P->p2 + 1) * (P->q + 1);
  const int ncell_max = column_cells(&c, c.sp1[0], c.sp2[0], NULL, NULL);
  const size_t per = 36 * (size_t)P->n_ply;
  double *part = (double *)calloc((size_t)c.ns2 * per, sizeof(double));
#pragma omp parallel
  {
    double (*grad)[3] = (double (*)[3])malloc(sizeof(double) * 3 * nloc);
    double (*Bm)[6][3] = (double (*)[6][3])malloc(sizeof(double) * 18 * nloc);
    double *Gl = (double *)malloc(sizeof(double) * 9 * (size_t)nloc * nloc);
    double (*V)[6][3] = (double (*)[6][3])malloc(sizeof(double) * 18 * nloc);
    int64_t *glob = (int64_t *)malloc(sizeof(int64_t) * nloc);
    cell_t *cells = (cell_t *)malloc(sizeof(cell_t) * (size_t)(ncell_max > 0 ? ncell_max : 1));
    int *plies = (int *)malloc(sizeof(int) * (size_t)(ncell_max > 0 ? ncell_max : 1));
#pragma omp for schedule(dynamic, 1)
    for (int z2 = 0; z2 < c.ns2; ++z2) {
      int s2 = c.sp2[z2];
      double *acc = part + (size_t)z2 * per;
      for (int z1 = 0; z1 < c.ns1; ++z1) {
        int s1 = c.sp1[z1];
        int ncell = column_cells(&c, s1, s2, cells, plies);
        for (int ic = 0; ic < ncell; ++ic) {
          const cell_t *cl = &cells[ic];
          double *dD = acc + 36 * (size_t)plies[ic];
          for (int a = 0; a < nloc; ++a) glob[a] = local_to_global(&c, cl, a);
          /* gather the local block of G */
          for (int a = 0; a < nloc; ++a)
            for (int r = 0; r < 3; ++r) {
              int64_t row = 3 * glob[a] + r;
              for (int b = 0; b < nloc; ++b)
                for (int s = 0; s < 3; ++s) {
                  int64_t pos = find_col(colind, rowptr[row], rowptr[row + 1], (int32_t)(3 * glob[b] + s));
                  Gl[((size_t)(3 * a + r)) * 3 * nloc + 3 * b + s] = G[pos];
                }
            }
          for (int g3 = 0; g3 < c.P.ngz; ++g3)
            for (int g2 = 0; g2 < c.P.ng2; ++g2)
              for (int g1 = 0; g1 < c.P.ng1; ++g1) {
                double R[256];
                double w = cell_point(&c, cl, g1, g2, g3, grad, R);
                for (int a = 0; a < nloc; ++a) bmat(grad[a], Bm[a]);
                /* V_a[J][r] = sum_{b,s} G[(a,r),(b,s)] B_b[J][s] */
                for (int a = 0; a < nloc; ++a)
                  for (int J = 0; J < 6; ++J)
                    for (int r = 0; r < 3; ++r) {
                      double t = 0.0;
                      for (int b = 0; b < nloc; ++b)
                        for (int s = 0; s < 3; ++s)
                          t += Gl[((size_t)(3 * a + r)) * 3 * nloc + 3 * b + s] * Bm[b][J][s];
                      V[a][J][r] = t;
                    }
                for (int I = 0; I < 6; ++I)
                  for (int J = 0; J < 6; ++J) {
                    double t = 0.0;
                    for (int a = 0; a < nloc; ++a)
                      for (int r = 0; r < 3; ++r) t += Bm[a][I][r] * V[a][J][r];
                    dD[I * 6 + J] += w * t;
                  }
              }
        }
      }
    }
    free(grad); free(Bm); free(Gl); free(V); free(glob); free(cells); free(plies);
  }
  for (size_t e = 0; e < per; ++e) dLdD[e] = 0.0;
  for (int z2 = 0; z2 < c.ns2; ++z2)
    for (size_t e = 0; e < per; ++e) dLdD[e] += part[(size_t)z2 * per + e];
  free(part);
  ctx_free(&c);
  return 0;
}

/* Chain rule from dL/dD_l to the material 6x6 matrices and the ply angles.
 * D_l is linear in C_{mat(l)}: dL/dC[K][L] = sum_l <dL/dD_l, D(E_KL, theta_l)>
 * with E_KL the unit 6x6; dL/dtheta_l = <dL/dD_l, dD/dtheta(C_{mat(l)}, theta_l)>. */
int or_grad_material(int32_t n_ply, const int32_t *ply_mat, const double *ply_theta, int32_t n_mat,
                     const double *C, const double *dLdD, double *gradC, double *gradTheta) {
  for (int e = 0; e < 36 * n_mat; ++e) gradC[e] = 0.0;
  for (int l = 0; l < n_ply; ++l) {
    int m = ply_mat[l];
    if (m < 0 || m >= n_mat) return -1;
    const double *M = dLdD + 36 * (size_t)l;
    for (int KL = 0; KL < 36; ++KL) {
      double E[36] = {0}, R[36];
      E[KL] = 1.0;
      or_rotate_voigt(E, ply_theta[l], R);
      double t = 0.0;
      for (int e = 0; e < 36; ++e) t += M[e] * R[e];
      gradC[36 * m + KL] += t;
    }
    double dD[36];
    or_rotate_voigt_dtheta(C + 36 * (size_t)m, ply_theta[l], dD);
    double t = 0.0;
    for (int e = 0; e < 36; ++e) t += M[e] * dD[e];
    gradTheta[l] = t;
  }
  return 0;
}

/* The mapped position of an in-plane parametric point and its two tangents:
 * S(xi1, xi2) = sum_i R^i ctrl_i and dS/dxi_k for a curved plan; for an
 * affine one, x = DF (xi1, xi2, 0) and the first two columns of DF. */
int or_surface_eval(const or_problem *P, double x1, double x2, double *x, double *t1, double *t2) {
  ctx c;
  if (ctx_init(&c, P)) { ctx_free(&c); return -1; }
  if (!(x1 >= 0.0 && x1 <= 1.0 && x2 >= 0.0 && x2 <= 1.0)) { ctx_free(&c); return -1; }
  for (int k = 0; k < 3; ++k) x[k] = t1[k] = t2[k] = 0.0;
  if (!P->ctrl) {
    for (int k = 0; k < 3; ++k) {
      x[k] = P->J[3 * k] * x1 + P->J[3 * k + 1] * x2;
      t1[k] = P->J[3 * k];
      t2[k] = P->J[3 * k + 1];
    }
    ctx_free(&c);
    return 0;
  }
  int s1 = find_span(P->p1, P->nk1, P->k1, x1), s2 = find_span(P->p2, P->nk2, P->k2, x2);
  double R[256], dR1[256], dR2[256];
  inplane_basis(&c, s1, s2, x1, x2, R, dR1, dR2);
  for (int b2 = 0; b2 <= P->p2; ++b2)
    for (int b1 = 0; b1 <= P->p1; ++b1) {
      int b = b2 * (P->p1 + 1) + b1;
      const double *X = P->ctrl + 3 * (size_t)((s2 - P->p2 + b2) * c.n1 + (s1 - P->p1 + b1));
      for (int k = 0; k < 3; ++k) {
        x[k] += R[b] * X[k];
        t1[k] += dR1[b] * X[k];
        t2[k] += dR2[b] * X[k];
      }
    }
  ctx_free(&c);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Plain definitions of the split operators of Sec. 3.
 *
 * P[alpha][beta][r][s] for in-plane functions (is, js) and a given 6x6 D
 * (eq. P): the 2D integral over the in-plane parametric domain of
 * B_alpha^{is T} D B_beta^{js} |DF|, where B_1 is built from
 * grad V = DF^{-T} (dS/dxi1, dS/dxi2, 0) and B_2 from W = DF^{-T} (0, 0, S). */
int or_P_pair(const or_problem *P, const double *D, int is, int js, double *Pout) {
  ctx c;
  if (ctx_init(&c, P)) { ctx_free(&c); return -1; }
  if (is < 0 || is >= c.ns || js < 0 || js >= c.ns) { ctx_free(&c); return -1; }
  int i1 = is % c.n1, i2 = is / c.n1, j1 = js % c.n1, j2 = js / c.n1;
  for (int e = 0; e < 36; ++e) Pout[e] = 0.0;
  for (int z2 = 0; z2 < c.ns2; ++z2) {
    int s2 = c.sp2[z2];
    if (s2 < i2 || s2 > i2 + P->p2 || s2 < j2 || s2 > j2 + P->p2) continue;
    for (int z1 = 0; z1 < c.ns1; ++z1) {
      int s1 = c.sp1[z1];
      if (s1 < i1 || s1 > i1 + P->p1 || s1 < j1 || s1 > j1 + P->p1) continue;
      for (int g2 = 0; g2 < c.P.ng2; ++g2)
        for (int g1 = 0; g1 < c.P.ng1; ++g1) {
          double x1, x2, h1, h2, R[256], dR1[256], dR2[256], Ji[9], det;
          point_coords(&c, s1, s2, g1, g2, &x1, &x2, &h1, &h2);
          inplane_basis(&c, s1, s2, x1, x2, R, dR1, dR2);
          point_geometry(&c, s1, s2, dR1, dR2, Ji, &det);
          double w = c.gw1[g1] * c.gw2[g2] * h1 * h2 * fabs(det);
          int bi = (i2 - (s2 - P->p2)) * (P->p1 + 1) + i1 - (s1 - P->p1);
          int bj = (j2 - (s2 - P->p2)) * (P->p1 + 1) + j1 - (s1 - P->p1);
          double hat[2][2][3]; /* [function i/j][alpha][component] */
          double gi[3] = {dR1[bi], dR2[bi], 0.0};
          double gj[3] = {dR1[bj], dR2[bj], 0.0};
          double wi[3] = {0.0, 0.0, R[bi]}, wj[3] = {0.0, 0.0, R[bj]};
          for (int k = 0; k < 3; ++k) {
            hat[0][0][k] = Ji[0 * 3 + k] * gi[0] + Ji[1 * 3 + k] * gi[1] + Ji[2 * 3 + k] * gi[2];
            hat[0][1][k] = Ji[0 * 3 + k] * wi[0] + Ji[1 * 3 + k] * wi[1] + Ji[2 * 3 + k] * wi[2];
            hat[1][0][k] = Ji[0 * 3 + k] * gj[0] + Ji[1 * 3 + k] * gj[1] + Ji[2 * 3 + k] * gj[2];
            hat[1][1][k] = Ji[0 * 3 + k] * wj[0] + Ji[1 * 3 + k] * wj[1] + Ji[2 * 3 + k] * wj[2];
          }
          for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be) {
              double Ba[6][3], Bb[6][3], blk[3][3];
              bmat(hat[0][al], Ba);
              bmat(hat[1][be], Bb);
              btdb(Ba, D, Bb, blk);
              for (int r = 0; r < 3; ++r)
                for (int s = 0; s < 3; ++s) Pout[((al * 2 + be) * 3 + r) * 3 + s] += w * blk[r][s];
            }
        }
    }
  }
  ctx_free(&c);
  return 0;
}

/* Q[alpha][beta] for thickness functions (it, jt) on ply l (eq. Q): the 1D
 * integral over the ply of tau_alpha^{it} tau_beta^{jt} with tau_1 = T and
 * tau_2 = dT/dxi3; alpha belongs to the test function it. */
int or_Q_pair(const or_problem *P, int ply, int it, int jt, double *Qout) {
  ctx c;
  if (ctx_init(&c, P)) { ctx_free(&c); return -1; }
  if (ply < 0 || ply >= P->n_ply || it < 0 || it >= c.nt || jt < 0 || jt >= c.nt) { ctx_free(&c); return -1; }
  for (int e = 0; e < 4; ++e) Qout[e] = 0.0;
  for (int z = 0; z < c.ns3; ++z) {
    int s3 = c.sp3[z];
    if (s3 < it || s3 > it + P->q || s3 < jt || s3 > jt + P->q) continue;
    double za = fmax(P->iface[ply], P->k3[s3]), zb = fmin(P->iface[ply + 1], P->k3[s3 + 1]);
    if (!(zb > za)) continue;
    double h = 0.5 * (zb - za);
    for (int g = 0; g < c.P.ngz; ++g) {
      double x = 0.5 * (za + zb) + h * c.gx3[g];
      double T[16], dT[16];
      bspline_on_span(P->q, P->k3, s3, x, T, dT);
      int ai = it - (s3 - P->q), aj = jt - (s3 - P->q);
      double ti[2] = {T[ai], dT[ai]}, tj[2] = {T[aj], dT[aj]};
      double w = c.gw3[g] * h;
      for (int al = 0; al < 2; ++al)
        for (int be = 0; be < 2; ++be) Qout[al * 2 + be] += w * ti[al] * tj[be];
    }
  }
  ctx_free(&c);
  return 0;
}

/* For L = u^T K u (G = u u^T), dL/dD_l = int_{ply l} eps(u) eps(u)^T |DF| dxi,
 * eps(u) = sum_a B_a u_a the Voigt strain of the discrete field (eq. Km_0 is
 * linear in D_l).  u holds 3 values per global function (DOF order). */
int or_grad_uu(const or_problem *P, const double *u, double *dLdD, int nthreads) {
  ctx c;
  if (P->mat_field || ctx_init(&c, P)) { if (!P->mat_field) ctx_free(&c); return -1; }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const int nloc = (P->p1 + 1) * (P->p2 + 1) * (P->q + 1);
  const int ncell_max = column_cells(&c, c.sp1[0], c.sp2[0], NULL, NULL);
  const size_t per = 36 * (size_t)P->n_ply;
  double *part = (double *)calloc((size_t)c.ns2 * per, sizeof(double));
#pragma omp parallel
  {
    double (*grad)[3] = (double (*)[3])malloc(sizeof(double) * 3 * nloc);
    cell_t *cells = (cell_t *)malloc(sizeof(cell_t) * (size_t)(ncell_max > 0 ? ncell_max : 1));
    int *plies = (int *)malloc(sizeof(int) * (size_t)(ncell_max > 0 ? ncell_max : 1));
#pragma omp for schedule(dynamic, 1)
    for (int z2 = 0; z2 < c.ns2; ++z2) {
      int s2 = c.sp2[z2];
      double *acc = part + (size_t)z2 * per;
      for (int z1 = 0; z1 < c.ns1; ++z1) {
        int s1 = c.sp1[z1];
        int ncell = column_cells(&c, s1, s2, cells, plies);
        for (int ic = 0; ic < ncell; ++ic) {
          const cell_t *cl = &cells[ic];
          double *dD = acc + 36 * (size_t)plies[ic];
          for (int g3 = 0; g3 < c.P.ngz; ++g3)
            for (int g2 = 0; g2 < c.P.ng2; ++g2)
              for (int g1 = 0; g1 < c.P.ng1; ++g1) {
                double R[256];
                double w = cell_point(&c, cl, g1, g2, g3, grad, R);
                double eps[6] = {0, 0, 0, 0, 0, 0};
                for (int a = 0; a < nloc; ++a) {
                  double B[6][3];
                  bmat(grad[a], B);
                  int64_t gi = local_to_global(&c, cl, a);
                  for (int I = 0; I < 6; ++I)
                    for (int r = 0; r < 3; ++r) eps[I] += B[I][r] * u[3 * gi + r];
                }
                for (int I = 0; I < 6; ++I)
                  for (int J = 0; J < 6; ++J) dD[I * 6 + J] += w * eps[I] * eps[J];
              }
        }
      }
    }
    free(grad); free(cells); free(plies);
  }
  for (size_t e = 0; e < per; ++e) dLdD[e] = 0.0;
  for (int z2 = 0; z2 < c.ns2; ++z2)
    for (size_t e = 0; e < per; ++e) dLdD[e] += part[(size_t)z2 * per + e];
  free(part);
  ctx_free(&c);
  return 0;
}
