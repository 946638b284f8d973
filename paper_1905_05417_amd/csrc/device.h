// device.h -- the device view of a plan and the device code that the
// single-laminate kernels (kernels.hip) and the batched ones (batch.hip)
// share: material rotation and bracket coefficients, the set checks, the 2D
// moments (affine and curved shells), the folded 1D coefficients and the
// register-mode scatter of one item.  One source for both paths.  Not part
// of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>

#include "internal.h"

namespace lamdev {

using lam::Region;

struct Dev {
  // sizes
  int p1, p2, q, n1, n2, nt, ns, ng1, ng2, ngz;
  int n_ply, n_mat, n_sets, set_mode, n_harm, maxact, n_tiles, tile_k;
  int64_t nnz2, nnzz, nnz, nrows;
  double jit[9], detj;
  // constant tables
  const double *tab1, *w1, *tab2, *w2;
  const int *e1first, *e2first;
  const int2 *pe1, *pe2;
  const int *srow, *krow, *kcol, *kp1, *kp2;
  const int *zfirst, *zply;
  const double *ztab, *zw;
  const int *zrow, *zcol, *zkrow, *zcptr, *zcell, *zaptr, *zaset;
  const int *set_mat, *set_aux, *ply_mat, *ply_set;
  const int *tiles, *chunk_ptr, *chunk_sptr, *chunk_set, *zaslot, *group_ptr, *group_sptr, *group_set, *chunk_lset;
  int n_chunks, chunk_sets, n_groups;
  int64_t kron_lds_q, kron_lds_p;
  const int *zchunk;
  int kron_nsc;
  const int *a1f, *a1c, *a2f, *a2c, *zs_first, *zs_cptr, *zs_cell;
  int ne1, ne2, nzs;
  double *Eply;
  const double *Escat;  // bracket coefficients of the scatter's sets: Ec, or Eply for harmonic plans
  int harm_ply;
  const int *rowply, *rowfin;
  double *Qp, *adj_part, *adj_y, *adj_cm;  // adj_cm: per ply, T^T dL/dD T (36)
  int *status;  // lam::N_STATUS flags, set by kernels, cleared by lam_check
  // curved shells: per-point map gradients and in-plane basis (constant);
  // material fields: set brackets per in-plane function and per point (scratch)
  int shell, mat_field, ngp, nb;
  const double *gtab, *rtab;
  double *Ectl, *Epts;
  // scratch
  double *D, *Ec, *P, *Qc, *M;
};

template <class T>
inline T *at(void *ws, const Region &r) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + r.off);
}

// Device view of a plan: constant tables (and status words) in the caller's
// workspace ws; the fast assembly's scratch regions [const_bytes, fwd_end) at
// sbase + (offset - const_bytes), by default right after the tables in ws.
// With an outside sbase (the static scratch of lam_assemble_static) the
// regions of the standard assembly and the adjoint are left null.
inline Dev make_dev(const lam_plan *p, void *ws, void *sbase = nullptr) {
  const bool own = sbase == nullptr;
  char *sb = (own ? static_cast<char *>(ws) + p->L.const_bytes : static_cast<char *>(sbase)) - p->L.const_bytes;
  Dev d;
  d.p1 = p->p1; d.p2 = p->p2; d.q = p->q;
  d.n1 = p->n1; d.n2 = p->n2; d.nt = p->nt; d.ns = p->ns;
  d.ng1 = p->ng1; d.ng2 = p->ng2; d.ngz = p->ngz;
  d.n_ply = p->n_ply; d.n_mat = p->n_mat; d.n_sets = p->n_sets; d.set_mode = p->set_mode;
  d.n_harm = p->n_harm; d.maxact = p->maxact; d.n_tiles = p->n_tiles; d.tile_k = p->tile_k;
  d.nnz2 = p->nnz2; d.nnzz = p->nnzz; d.nnz = p->nnz; d.nrows = p->nrows;
  for (int a = 0; a < 9; ++a) d.jit[a] = p->jit[a];
  d.detj = p->detj;
  const lam::Layout &L = p->L;
  d.tab1 = at<double>(ws, L.tab1); d.w1 = at<double>(ws, L.w1);
  d.tab2 = at<double>(ws, L.tab2); d.w2 = at<double>(ws, L.w2);
  d.e1first = at<int>(ws, L.e1first); d.e2first = at<int>(ws, L.e2first);
  d.pe1 = at<int2>(ws, L.pe1); d.pe2 = at<int2>(ws, L.pe2);
  d.srow = at<int>(ws, L.srow); d.krow = at<int>(ws, L.krow); d.kcol = at<int>(ws, L.kcol);
  d.kp1 = at<int>(ws, L.kp1); d.kp2 = at<int>(ws, L.kp2);
  d.zfirst = at<int>(ws, L.zfirst); d.zply = at<int>(ws, L.zply);
  d.ztab = at<double>(ws, L.ztab); d.zw = at<double>(ws, L.zw);
  d.zrow = at<int>(ws, L.zrow); d.zcol = at<int>(ws, L.zcol); d.zkrow = at<int>(ws, L.zkrow);
  d.zcptr = at<int>(ws, L.zcptr); d.zcell = at<int>(ws, L.zcell);
  d.zaptr = at<int>(ws, L.zaptr); d.zaset = at<int>(ws, L.zaset);
  d.set_mat = at<int>(ws, L.set_mat); d.set_aux = at<int>(ws, L.set_aux);
  d.ply_mat = at<int>(ws, L.ply_mat); d.ply_set = at<int>(ws, L.ply_set);
  d.tiles = at<int>(ws, L.tiles);
  d.chunk_ptr = at<int>(ws, L.chunk_ptr);
  d.chunk_sptr = at<int>(ws, L.chunk_sptr);
  d.chunk_set = at<int>(ws, L.chunk_set);
  d.zaslot = at<int>(ws, L.zaslot);
  d.n_chunks = p->n_chunks;
  d.group_ptr = at<int>(ws, L.group_ptr);
  d.group_sptr = at<int>(ws, L.group_sptr);
  d.group_set = at<int>(ws, L.group_set);
  d.chunk_lset = at<int>(ws, L.chunk_lset);
  d.n_groups = p->n_groups;
  d.chunk_sets = p->chunk_sets;
  d.kron_lds_q = p->kron_lds_q;
  d.zchunk = at<int>(ws, L.zchunk);
  d.a1f = at<int>(ws, L.a1f); d.a1c = at<int>(ws, L.a1c);
  d.a2f = at<int>(ws, L.a2f); d.a2c = at<int>(ws, L.a2c);
  d.zs_first = at<int>(ws, L.zs_first); d.zs_cptr = at<int>(ws, L.zs_cptr); d.zs_cell = at<int>(ws, L.zs_cell);
  d.ne1 = p->ne1; d.ne2 = p->ne2; d.nzs = p->nzs;
  d.Eply = at<double>(sb, L.Eply);
  d.harm_ply = p->harm_ply;
  d.rowply = at<int>(ws, L.rowply); d.rowfin = at<int>(ws, L.rowfin);
  d.Qp = own ? at<double>(sb, L.Qp) : nullptr;
  d.adj_part = own ? at<double>(sb, L.adj_part) : nullptr;
  d.adj_y = own ? at<double>(sb, L.adj_y) : nullptr;
  d.adj_cm = own ? at<double>(sb, L.adj_cm) : nullptr;
  d.kron_nsc = p->kron_nsc;
  d.kron_lds_p = p->kron_lds_p;
  d.status = at<int>(ws, L.status);
  d.shell = p->shell;
  d.mat_field = p->mat_field;
  d.ngp = p->ng1 * p->ng2;
  d.nb = (p->p1 + 1) * (p->p2 + 1);
  d.gtab = at<double>(ws, L.gtab);
  d.rtab = at<double>(ws, L.rtab);
  d.Ectl = at<double>(sb, L.Ectl);
  d.Epts = at<double>(sb, L.Epts);
  d.D = at<double>(sb, L.D); d.Ec = at<double>(sb, L.Ec); d.P = at<double>(sb, L.P);
  d.Escat = p->harm_ply ? d.Eply : d.Ec;
  d.Qc = at<double>(sb, L.Qc); d.M = at<double>(sb, L.M);
  return d;
}

// ---------------------------------------------------------------------------
// Material rotation (eq. D).  With R[i][k] = e_i . a_k (material axes
// a_1 = (c,s,0), a_2 = (-s,c,0), a_3 = e_3), the Voigt stress transformation
// is T[I][J] = R[i][k] R[j][l] + [k != l] R[i][l] R[j][k] for I = (ij),
// J = (kl); engineering strains transform with T^T, so D = T C T^T.
static __constant__ int kVi[6] = {0, 1, 2, 0, 0, 1};
static __constant__ int kVj[6] = {0, 1, 2, 1, 2, 2};

// Layout of the moments M_ab[kl] (36 per in-plane nonzero k, e = 9 ab + kl):
// blocks of 64 consecutive nonzeros, each holding the 36 arrays of its 64
// values.  A scatter tile (a run of about 64 consecutive nonzeros) reads one
// or two contiguous 18 KB runs, coalesced across its lanes, instead of 36
// runs nnz2 values apart (36 pages per block on the large plates).
__device__ inline int64_t m_index(int64_t k, int e) { return (k >> 6) * (36 * 64) + e * 64 + (k & 63); }

__device__ inline void voigt_rotation(double c, double s, double T[6][6]) {
  const double R[3][3] = {{c, -s, 0.0}, {s, c, 0.0}, {0.0, 0.0, 1.0}};
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      int i = kVi[I], j = kVj[I], k = kVi[J], l = kVj[J];
      double t = R[i][k] * R[j][l];
      if (k != l) t += R[i][l] * R[j][k];
      T[I][J] = t;
    }
}

__device__ inline void rotate_c(const double *C, double c, double s, double D[6][6]) {
  double T[6][6], TC[6][6];
  voigt_rotation(c, s, T);
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      double a = 0.0;
      for (int K = 0; K < 6; ++K) a += T[I][K] * C[K * 6 + J];
      TC[I][J] = a;
    }
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      double a = 0.0;
      for (int K = 0; K < 6; ++K) a += TC[I][K] * T[J][K];
      D[I][J] = a;
    }
}

// Harmonic h of a set: order and kind (0 constant, 1 cosine, 2 sine).
__device__ inline void harmonic(int n_harm, int h, int &order, int &kind) {
  if (h == 0) { order = 0; kind = 0; return; }
  if (n_harm == 5) { order = 2 * ((h + 1) / 2); kind = (h & 1) ? 1 : 2; return; }
  order = (h + 1) / 2;
  kind = (h & 1) ? 1 : 2;
}

__device__ inline double harmonic_weight(int n_harm, int h, double theta) {
  int order, kind;
  harmonic(n_harm, h, order, kind);
  if (kind == 0) return 1.0;
  return kind == 1 ? cos(order * theta) : sin(order * theta);
}

// Voigt strain of the displacement e_r * phi for a unit gradient e_k:
// column r of B(e_k) (eq. B_1 with the gamma_23 entry of the u_3 column
// taking the 2-derivative).
__device__ inline double bunit(int k, int I, int r) {
  // B(g)[I][r]: rows 11,22,33,12,13,23
  switch (I) {
    case 0: return (r == 0 && k == 0) ? 1.0 : 0.0;
    case 1: return (r == 1 && k == 1) ? 1.0 : 0.0;
    case 2: return (r == 2 && k == 2) ? 1.0 : 0.0;
    case 3: return ((r == 0 && k == 1) || (r == 1 && k == 0)) ? 1.0 : 0.0;
    case 4: return ((r == 0 && k == 2) || (r == 2 && k == 0)) ? 1.0 : 0.0;
    default: return ((r == 1 && k == 2) || (r == 2 && k == 1)) ? 1.0 : 0.0;
  }
}

// E[k][l][r][t] = sum_IJ B(e_k)[I][r] D[I][J] B(e_l)[J][t]: the 3x3 block
// B(a)^T D B(b) of two gradients is sum_kl a_k b_l E[k][l].
__device__ inline void bracket_coefficients(const double D[6][6], double *E) {
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l)
      for (int r = 0; r < 3; ++r)
        for (int t = 0; t < 3; ++t) {
          double a = 0.0;
          for (int I = 0; I < 6; ++I) {
            double bi = bunit(k, I, r);
            if (bi == 0.0) continue;
            for (int J = 0; J < 6; ++J) a += bi * D[I][J] * bunit(l, J, t);
          }
          E[((k * 3 + l) * 3 + r) * 3 + t] = a;
        }
}

// One thread per set.  Harmonic sets: the Fourier coefficient of D(phi)
// sampled at NH equispaced angles (exact for trigonometric polynomials of
// degree <= 4 once NH >= 9).
constexpr int NH = 12;

// Inputs a plan cannot honour raise a status word (plain stores of 1, never
// cleared here; lam_check reads and clears them):
//  - bucket sets: a ply given another angle than its set's first ply (the set
//    is rotated by that one angle, so K would not be K(theta));
//  - harmonic5 sets: a material with a nonzero {11,22,33,12}-{13,23} entry
//    (relative to its largest entry, above 1e-13), whose rotation has odd
//    harmonics that five terms do not hold (Remark on orientations).
// (the bucket check runs per ply, check_ply; the harmonic5 one per material)
__device__ __forceinline__ void check_ply(const Dev &d, const double *__restrict__ theta, int l) {
  if (d.set_mode == LAM_SETS_BUCKET && l < d.n_ply && !(theta[l] == theta[d.set_aux[d.ply_set[l]]])) d.status[0] = 1;
}

__device__ __forceinline__ void check_set(const Dev &d, const double *__restrict__ Cm, int s) {
  if (d.set_mode != LAM_SETS_BUCKET && d.n_harm == 5 && d.set_aux[s] == 0) {
    double big = 0.0, cpl = 0.0;
    for (int e = 0; e < 36; ++e) big = fmax(big, fabs(Cm[e]));
    for (int I = 0; I < 4; ++I)
      for (int J = 4; J < 6; ++J) cpl = fmax(cpl, fmax(fabs(Cm[6 * I + J]), fabs(Cm[6 * J + I])));
    if (!(cpl <= 1e-13 * big)) d.status[1] = 1;
  }
}

__device__ __forceinline__ void rotate_one(const Dev &d, const double *__restrict__ C, const double *__restrict__ theta,
                                           int s) {
  if (s >= d.n_sets) return;
  const double *Cm = C + 36 * d.set_mat[s];
  check_set(d, Cm, s);
  double D[6][6];
  if (d.set_mode == LAM_SETS_BUCKET) {
    double th = theta[d.set_aux[s]];
    rotate_c(Cm, cos(th), sin(th), D);
  } else {
    int order, kind;
    harmonic(d.n_harm, d.set_aux[s], order, kind);
    for (int I = 0; I < 6; ++I)
      for (int J = 0; J < 6; ++J) D[I][J] = 0.0;
    for (int j = 0; j < NH; ++j) {
      double phi = 2.0 * M_PI * j / NH;
      double wgt = kind == 0 ? 1.0 / NH : (kind == 1 ? 2.0 * cos(order * phi) : 2.0 * sin(order * phi)) / NH;
      double Dj[6][6];
      rotate_c(Cm, cos(phi), sin(phi), Dj);
      for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) D[I][J] += wgt * Dj[I][J];
    }
  }
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) d.D[36 * s + 6 * I + J] = D[I][J];
  bracket_coefficients(D, d.Ec + 81 * s);
}

// 1D moments of functions i and j of one in-plane direction over the elements
// of their common support (range: first element, count), by Gauss quadrature:
// out = {int N_i N_j, int N_i' N_j, int N_i N_j', int N_i' N_j'} (weights include
// the element length).
__device__ __forceinline__ void moments_1d(const double *__restrict__ tab, const double *__restrict__ w,
                                           const int *__restrict__ efirst, int2 range, int ng, int P, int i, int j,
                                           double out[4]) {
  out[0] = out[1] = out[2] = out[3] = 0.0;
  for (int e = range.x; e < range.x + range.y; ++e) {
    const int f = efirst[e];
    const int ai = i - f, aj = j - f;
    for (int g = 0; g < ng; ++g) {
      const double *t = tab + ((int64_t)e * ng + g) * P * 2;
      const double Ni = t[2 * ai], dNi = t[2 * ai + 1], Nj = t[2 * aj], dNj = t[2 * aj + 1];
      const double wg = w[(int64_t)e * ng + g];
      out[0] += wg * Ni * Nj;
      out[1] += wg * dNi * Nj;
      out[2] += wg * Ni * dNj;
      out[3] += wg * dNi * dNj;
    }
  }
}

// ---------------------------------------------------------------------------
// 2D operators (eq. P).  For in-plane pair k = (is, js), the 2D Gauss sum
// over the elements shared by both supports of the parametric moments
//   m11[a][b] = sum w dS^i/dxi_a dS^j/dxi_b,  m12[a] = sum w dS^i/dxi_a S^j,
//   m21[b]    = sum w S^i dS^j/dxi_b,         m22    = sum w S^i S^j,
// pushed through DF^{-T} (grad V = DF^{-T}(dS1,dS2,0), W = DF^{-T}(0,0,S))
// into M_ab[k][l] = int (G_a^i)_k (G_b^j)_l |DF|.  Because each set's
// material is constant over the plane, P_{s,ab}[r][t] = sum_kl M_ab[k][l] E_s[k][l][r][t].
__device__ __forceinline__ void affine_moments(const Dev &d, int64_t k, double (&M)[4][3][3]) {
  const int is = d.krow[k], js = d.kcol[k];
  const int i1 = is % d.n1, i2 = is / d.n1, j1 = js % d.n1, j2 = js / d.n1;
  const int2 ra = d.pe1[d.kp1[k]], rb = d.pe2[d.kp2[k]];
  const int P1 = d.p1 + 1, P2 = d.p2 + 1;
  // The in-plane map is affine (eq. extrusion) and the basis a tensor product
  // (eq. basis_functions), and the 2D Gauss rule is a tensor product too, so
  // each parametric moment of eq. P is exactly a product of two 1D moments:
  // u of direction 1, v of direction 2, each {int N_i N_j, int N_i' N_j,
  // int N_i N_j', int N_i' N_j'} over the common support.
  double u[4], v[4];
  moments_1d(d.tab1, d.w1, d.e1first, ra, d.ng1, P1, i1, j1, u);
  moments_1d(d.tab2, d.w2, d.e2first, rb, d.ng2, P2, i2, j2, v);
  double m11[2][2], m12[2], m21[2];
  m11[0][0] = u[3] * v[0];
  m11[0][1] = u[1] * v[2];
  m11[1][0] = u[2] * v[1];
  m11[1][1] = u[0] * v[3];
  m12[0] = u[1] * v[0];
  m12[1] = u[0] * v[1];
  m21[0] = u[2] * v[0];
  m21[1] = u[0] * v[2];
  const double m22 = u[0] * v[0];
  // M_ab[k][l], ab = 11, 12, 21, 22
  const double *J = d.jit;
#pragma unroll
  for (int kk = 0; kk < 3; ++kk)
#pragma unroll
    for (int ll = 0; ll < 3; ++ll) {
      double v11 = 0.0, v12 = 0.0, v21 = 0.0;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        v12 += J[kk * 3 + a] * m12[a];
        v21 += J[ll * 3 + a] * m21[a];
#pragma unroll
        for (int b = 0; b < 2; ++b) v11 += J[kk * 3 + a] * J[ll * 3 + b] * m11[a][b];
      }
      M[0][kk][ll] = d.detj * v11;
      M[1][kk][ll] = d.detj * v12 * J[ll * 3 + 2];
      M[2][kk][ll] = d.detj * J[kk * 3 + 2] * v21;
      M[3][kk][ll] = d.detj * J[kk * 3 + 2] * J[ll * 3 + 2] * m22;
    }
}

// The same moments on a curved shell (Assumption 2 with a curved mid-surface,
// eq. extrusion): DF^{-T} and |DF| change from point to point and the basis may
// be rational, so the moments are plain 2D Gauss sums over the shared
// elements, M_ab[k][l] = sum_e sum_g w |DF| (G_a^i)_k (G_b^j)_l with
// G_1 = DF^{-T} (dR/dxi1, dR/dxi2, 0) and G_2 = DF^{-T} (0, 0, R) (eq. B_2).
__device__ __forceinline__ void shell_moments(const Dev &d, int64_t k, double (&M)[4][3][3]) {
  const int is = d.krow[k], js = d.kcol[k];
  const int i1 = is % d.n1, i2 = is / d.n1, j1 = js % d.n1, j2 = js / d.n1;
  const int2 ra = d.pe1[d.kp1[k]], rb = d.pe2[d.kp2[k]];
  const int P1 = d.p1 + 1;
#pragma unroll
  for (int ab = 0; ab < 4; ++ab)
#pragma unroll
    for (int e = 0; e < 9; ++e) M[ab][e / 3][e % 3] = 0.0;
  for (int e2 = rb.x; e2 < rb.x + rb.y; ++e2) {
    const int f2 = d.e2first[e2];
    for (int e1 = ra.x; e1 < ra.x + ra.y; ++e1) {
      const int f1 = d.e1first[e1];
      const int64_t e = e1 + (int64_t)d.ne1 * e2;
      const int bi = (i2 - f2) * P1 + (i1 - f1), bj = (j2 - f2) * P1 + (j1 - f1);
      for (int g = 0; g < d.ngp; ++g) {
        const double *G = d.gtab + (e * d.ngp + g) * 10;
        const double *ri = d.rtab + ((e * d.ngp + g) * d.nb + bi) * 3;
        const double *rj = d.rtab + ((e * d.ngp + g) * d.nb + bj) * 3;
        double vi[2][3], vj[2][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          vi[0][c] = G[c * 3] * ri[1] + G[c * 3 + 1] * ri[2];
          vi[1][c] = G[c * 3 + 2] * ri[0];
          vj[0][c] = G[c * 3] * rj[1] + G[c * 3 + 1] * rj[2];
          vj[1][c] = G[c * 3 + 2] * rj[0];
        }
        const double w = G[9];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
#pragma unroll
          for (int ll = 0; ll < 3; ++ll) {
            M[0][kk][ll] += w * vi[0][kk] * vj[0][ll];
            M[1][kk][ll] += w * vi[0][kk] * vj[1][ll];
            M[2][kk][ll] += w * vi[1][kk] * vj[0][ll];
            M[3][kk][ll] += w * vi[1][kk] * vj[1][ll];
          }
      }
    }
  }
}

__device__ __forceinline__ void p2d_one(const Dev &d, const double *__restrict__ Ec, double *__restrict__ Pt,
                                        double *__restrict__ Mt, int64_t k, int write_p) {
  if (k >= d.nnz2) return;
  double M[4][3][3];
  if (d.shell)
    shell_moments(d, k, M);
  else
    affine_moments(d, k, M);
  // component-major tables: consecutive threads (k) store consecutive addresses
#pragma unroll
  for (int ab = 0; ab < 4; ++ab)
#pragma unroll
    for (int e = 0; e < 9; ++e) Mt[m_index(k, ab * 9 + e)] = M[ab][e / 3][e % 3];
  for (int s = 0; s < (write_p ? d.n_sets : 0); ++s) {
    const double *E = Ec + 81 * s;
    double *Po = Pt + (int64_t)s * 36 * d.nnz2 + k;
#pragma unroll
    for (int ab = 0; ab < 4; ++ab)
#pragma unroll
      for (int rt = 0; rt < 9; ++rt) {
        double a = 0.0;
#pragma unroll
        for (int kl = 0; kl < 9; ++kl) a += M[ab][kl / 3][kl % 3] * E[kl * 9 + rt];
        Po[(int64_t)(ab * 9 + rt) * d.nnz2] = a;
      }
  }
}


// ---------------------------------------------------------------------------
// 1D operators (eq. Q) folded into the sets: for thickness pair zk = (it, jt)
// and the j-th set active on row it,
//   Qc[zk][j][ab] = sum_{cells c shared by it, jt} w_{s,ply(c)} sum_g w_g tau_a^{it} tau_b^{jt}
// with tau_1 = T, tau_2 = dT/dxi3, a on the test function it, and
// w_{s,l} = [set of l == s] (bucket) or [mat(l) == mat(s)] * harmonic_s(theta_l).
// One wave per entry (thickness nonzero zk, set slot j): the lanes split the
// cells the pair shares (with one thickness element through many plies every
// ply is such a cell, so a single thread would sum m (q+1) terms in turn) and
// a fixed butterfly over the wave adds the lanes' sums (deterministic).
__device__ __forceinline__ void q1d_wave(const Dev &d, const double *__restrict__ theta, int64_t idx, int lane) {
  // register mode: one entry per chunk set slot (zeros where the slot's set
  // does not act on the pair); LDS mode: one per set active on the row
  const int width = d.kron_nsc > 0 ? d.kron_nsc : d.maxact;
  if (idx >= d.nnzz * width) return;  // uniform over the wave
  const int zk = (int)(idx / width), j = (int)(idx % width);
  const int it = d.zkrow[zk], jt = d.zcol[zk];
  int s = -1;
  if (d.kron_nsc > 0) {
    const int ch = d.zchunk[it], c0 = d.chunk_sptr[ch];
    if (j < d.chunk_sptr[ch + 1] - c0) s = d.chunk_set[c0 + j];
  } else {
    const int a0 = d.zaptr[it];
    if (j < d.zaptr[it + 1] - a0) s = d.zaset[a0 + j];
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (s >= 0) {
    const int Q1 = d.q + 1;
    for (int ci = d.zcptr[zk] + lane; ci < d.zcptr[zk + 1]; ci += 64) {
      const int c = d.zcell[ci], l = d.zply[c];
      double wgt;
      if (d.harm_ply) {
        wgt = l == s ? 1.0 : 0.0;  // the scatter's sets are the plies
      } else if (d.set_mode == LAM_SETS_BUCKET) {
        wgt = d.ply_set[l] == s ? 1.0 : 0.0;
      } else {
        wgt = d.ply_mat[l] == d.set_mat[s] ? harmonic_weight(d.n_harm, d.set_aux[s], theta[l]) : 0.0;
      }
      if (wgt == 0.0) continue;
      const int ai = it - d.zfirst[c], aj = jt - d.zfirst[c];
      double q11 = 0.0, q12 = 0.0, q21 = 0.0, q22 = 0.0;
      for (int g = 0; g < d.ngz; ++g) {
        const double *t = d.ztab + ((int64_t)c * d.ngz + g) * Q1 * 2;
        const double Ti = t[2 * ai], dTi = t[2 * ai + 1], Tj = t[2 * aj], dTj = t[2 * aj + 1];
        const double w = d.zw[(int64_t)c * d.ngz + g];
        q11 += w * Ti * Tj;
        q12 += w * Ti * dTj;
        q21 += w * dTi * Tj;
        q22 += w * dTi * dTj;
      }
      acc[0] += wgt * q11;
      acc[1] += wgt * q12;
      acc[2] += wgt * q21;
      acc[3] += wgt * q22;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e] += __shfl_xor(acc[e], off, 64);
  if (lane == 0) {
    double *o = d.Qc + 4 * idx;
    o[0] = acc[0];
    o[1] = acc[1];
    o[2] = acc[2];
    o[3] = acc[3];
  }
}


constexpr int KRON_THREADS = 256;  // 3 * tile_k <= KRON_THREADS
constexpr int KRON_AB = 5;         // thickness columns per register block


// One thickness row of the register-mode scatter with its width LZ known at
// compile time (no per-column predicates): value (x, r) = sum over the
// chunk's set slots u of Qd[zk + x][u][ab] * P_u[ab][r] (eq. Km_2), the first
// slot's product starting the sum; stores r-major, x-minor.
template <int NSC, int LZ, class QP>
__device__ __forceinline__ void kron_row(QP qq, const double (&pr)[NSC][4][3], double *out, int64_t rstride,
                                         int64_t astride) {
  double acc[LZ][3];
  // slot-outer: one slot's coefficients of every column are read together
#pragma unroll
  for (int u = 0; u < NSC; ++u) {
    double qv[LZ][4];
#pragma unroll
    for (int x = 0; x < LZ; ++x)
#pragma unroll
      for (int ab = 0; ab < 4; ++ab) qv[x][ab] = qq[4 * NSC * x + 4 * u + ab];
#pragma unroll
    for (int x = 0; x < LZ; ++x)
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double v = qv[x][0] * pr[u][0][r] + qv[x][1] * pr[u][1][r] + qv[x][2] * pr[u][2][r] + qv[x][3] * pr[u][3][r];
        acc[x][r] = u == 0 ? v : acc[x][r] + v;
      }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int x = 0; x < LZ; ++x) out[r * rstride + (int64_t)x * astride] = acc[x][r];
}

// A value that is the same for the whole block, read from a plan table (the
// tables are written before any launch and only read while kernels run)
// through the constant address space: a scalar load, counted apart from the
// vector memory operations (whose counter includes the stores in flight), also
// where the compiler cannot see that the table is unwritten (the batch reads
// its per-laminate views from memory).
__device__ __forceinline__ int uld(const int *p, int64_t i) {
  return reinterpret_cast<const __attribute__((address_space(4))) int *>(reinterpret_cast<uintptr_t>(p))[i];
}

// Register-mode scatter of one (tile of whole in-plane rows, group of
// consecutive thickness chunks) item with one or two set slots per chunk (every
// bucket and per-ply plan): the block stages the bracket coefficients of the
// group's sets in LDS behind one barrier; then per chunk each thread (in-plane
// nonzero k, component t) contracts P of the chunk's slots from the
// set-independent moments M_ab[kl] and the slot's brackets E_s[kl][rt] (eq. P;
// P is never stored; material-field plans load their stored P instead) and
// writes the chunk's rows.  A row's slot-dense coefficients Qd[zk][slot][ab]
// are the same for the whole block: they are read from global memory through
// the constant address space, i.e. by scalar loads into scalar registers (also
// for the batch, whose qd comes from a per-laminate table), which keeps them
// out of the vector registers and, as scalar loads are counted apart from
// vector memory operations, waits on no store in flight; a row's are read slot
// by slot, all columns of a slot together, and its end index a row ahead, so
// that a row waits on one scalar load round trip.  After the barrier the block issues no vector load (constant materials): a
// vector load on any path into the row loop would make every row wait for all
// of the wave's stores in flight (loads and stores share one counter on this
// chip).  FIELD (material fields), a separate instantiation: each slot's P is
// read from the stored P of its set, at every set change.
// Block-cooperative: every thread of the block calls it with the same item
// (it holds a barrier; threads past 3 * tile_k return after it).  lq: LDS of
// kron_lds_q bytes (not used here; the matrix-free product stages its
// coefficients there), then 81 doubles per set of the group and 81 zeros.  The single-laminate scatter and the
// batched one both run it.
template <int NSC, bool FIELD>
__device__ __forceinline__ void kron_group(const Dev &d, const double *__restrict__ qd, double *__restrict__ vals,
                                           int tile, int g, double *lq, int sig, int nthreads) {
  static_assert(NSC <= 2, "grouped scatter items keep at most two set slots");
  const int k0 = uld(d.tiles, tile), tk = uld(d.tiles, tile + 1) - k0;
  const bool act = sig < 3 * tk;
  const int kk = act ? sig / 3 : 0, t = act ? sig - 3 * kk : 0, k = k0 + kk;
  double mv[4][9];  // the moments (material fields read their stored P instead)
  if constexpr (!FIELD) {
#pragma unroll
    for (int ab = 0; ab < 4; ++ab)
#pragma unroll
      for (int kl = 0; kl < 9; ++kl) mv[ab][kl] = d.M[m_index(k, ab * 9 + kl)];
  }
  const int is = d.krow[k], sr = d.srow[is];
  const int Ls = d.srow[is + 1] - sr, off = 3 * (k - sr) + t;
  const int64_t astride = 3 * (int64_t)Ls;
  double *le = lq + d.kron_lds_q / 8;
  const int ch0 = uld(d.group_ptr, g), ch1 = uld(d.group_ptr, g + 1);
  const int s0 = uld(d.group_sptr, g), ns = uld(d.group_sptr, g + 1) - s0;
  for (int e = sig; e < 81 * (ns + 1); e += nthreads) {
    const int u = e / 81;
    le[e] = u < ns ? d.Escat[81 * (int64_t)uld(d.group_set, s0 + u) + (e - 81 * u)] : 0.0;
  }
  __syncthreads();
  if (!act) return;  // no barrier follows
  double pr[NSC][4][3];
  int slot_set[NSC];  // group-local set of each slot's P
#pragma unroll
  for (int u = 0; u < NSC; ++u) slot_set[u] = -1;
  for (int ch = ch0; ch < ch1; ++ch) {
    const int it0 = uld(d.chunk_ptr, ch), it1 = uld(d.chunk_ptr, ch + 1);
    const int c0 = uld(d.chunk_sptr, ch), nsc = uld(d.chunk_sptr, ch + 1) - c0;
#pragma unroll
    for (int u = 0; u < NSC; ++u) {
      const int ls = u < nsc ? uld(d.chunk_lset, c0 + u) : ns;  // unused slots: the zero block
      if (ls == slot_set[u]) continue;  // the slot keeps its set (and P) from the previous chunk
      slot_set[u] = ls;
      if constexpr (FIELD) {  // P of the slot's set from memory (zero for an unused slot)
        const int gs = ls < ns ? uld(d.group_set, s0 + ls) : -1;
#pragma unroll
        for (int ab = 0; ab < 4; ++ab)
#pragma unroll
          for (int r = 0; r < 3; ++r)
            pr[u][ab][r] = gs >= 0 ? d.P[((int64_t)gs * 36 + ab * 9 + 3 * r + t) * d.nnz2 + k] : 0.0;
        continue;
      }
      const double *eu = le + 81 * ls;
#pragma unroll
      for (int ab = 0; ab < 4; ++ab)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          double a = 0.0;
#pragma unroll
          for (int kl = 0; kl < 9; ++kl) a += mv[ab][kl] * eu[kl * 9 + 3 * r + t];
          pr[u][ab][r] = a;
        }
    }
    int zb = uld(d.zrow, it0), zn = uld(d.zrow, it0 + 1);
    for (int it = it0; it < it1; ++it) {
      // the next row's end, read a row ahead (zrow has nt + 1 entries)
      const int zn2 = uld(d.zrow, it + 2 <= d.nt ? it + 2 : d.nt);
      const int Lz = zn - zb;
      double *out = vals + 9 * d.nnz2 * (int64_t)zb + 9 * (int64_t)Lz * sr + off;
      const int64_t rstride = 3 * (int64_t)Lz * Ls;
      // the row's coefficients, uniform over the block: scalar loads through
      // the constant address space (they do not wait on the stores in flight)
      const auto qz =
          reinterpret_cast<const __attribute__((address_space(4))) double *>(reinterpret_cast<uintptr_t>(qd)) +
          4 * NSC * (int64_t)zb;
      switch (Lz) {  // widths 2..5 (q + 1 up to q = 4, 2q + 1 up to q = 2) fixed; 7 and 9 take the loop
        case 2: kron_row<NSC, 2>(qz, pr, out, rstride, astride); break;
        case 3: kron_row<NSC, 3>(qz, pr, out, rstride, astride); break;
        case 4: kron_row<NSC, 4>(qz, pr, out, rstride, astride); break;
        case 5: kron_row<NSC, 5>(qz, pr, out, rstride, astride); break;
        default:
          for (int ab0 = 0; ab0 < Lz; ab0 += KRON_AB) {
            double acc[KRON_AB][3];
#pragma unroll
            for (int x = 0; x < KRON_AB; ++x) {
              acc[x][0] = acc[x][1] = acc[x][2] = 0.0;
              if (ab0 + x < Lz) {
                const auto qq = qz + 4 * NSC * (ab0 + x);
#pragma unroll
                for (int u = 0; u < NSC; ++u) {
                  const double q0 = qq[4 * u], q1 = qq[4 * u + 1], q2 = qq[4 * u + 2], q3 = qq[4 * u + 3];
#pragma unroll
                  for (int r = 0; r < 3; ++r)
                    acc[x][r] += q0 * pr[u][0][r] + q1 * pr[u][1][r] + q2 * pr[u][2][r] + q3 * pr[u][3][r];
                }
              }
            }
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
              for (int x = 0; x < KRON_AB; ++x)
                if (ab0 + x < Lz) out[r * rstride + (int64_t)(ab0 + x) * astride] = acc[x][r];
          }
      }
      zb = zn;
      zn = zn2;
    }
  }
}

}  // namespace lamdev
