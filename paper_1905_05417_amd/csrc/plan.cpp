// plan.cpp -- host side of the C ABI: descriptor validation, knot spans,
// basis tables at Gauss points, the in-plane / thickness / Kronecker CSR
// structure, the grouping of plies into sets, and the workspace layout.
//
// Everything here depends only on the discretisation (knots, plies, Gauss
// rules), never on the material values or angles, which arrive on the device
// at assembly time.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "internal.h"

namespace {

using lam::MAXG;
using lam::MAXP;

// Gauss-Legendre nodes/weights on [-1,1]: Newton's method on P_n from the
// asymptotic first guess, derivative from P'_n = n (x P_n - P_{n-1}) / (x^2 - 1).
void gauss_rule(int n, double *x, double *w) {
  const double pi = 3.141592653589793238462643;
  for (int k = 1; k <= n; ++k) {
    double t = std::cos(pi * (4.0 * k - 1.0) / (4.0 * n + 2.0));
    double pn = 0, pm = 0;
    for (int it = 0; it < 64; ++it) {
      pm = 1.0;
      pn = t;
      for (int j = 2; j <= n; ++j) {
        double pj = ((2 * j - 1) * t * pn - (j - 1) * pm) / j;
        pm = pn;
        pn = pj;
      }
      if (n == 1) { pm = 1.0; pn = t; }
      double dp = n * (t * pn - pm) / (t * t - 1.0);
      double step = pn / dp;
      t -= step;
      if (std::fabs(step) <= 1e-17) break;
    }
    pm = 1.0;
    pn = t;
    for (int j = 2; j <= n; ++j) {
      double pj = ((2 * j - 1) * t * pn - (j - 1) * pm) / j;
      pm = pn;
      pn = pj;
    }
    double dp = (n == 1) ? 1.0 : n * (t * pn - pm) / (t * t - 1.0);
    // t runs from the largest root down; store ascending
    x[n - k] = t;
    w[n - k] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  if (n & 1) x[n / 2] = 0.0;
}

// Values and first derivatives of the p+1 B-splines nonzero on knot span s
// (t[s] <= u < t[s+1]), by de Boor's left/right differences.
void basis_and_derivative(int p, const double *t, int s, double u, double *val, double *der) {
  double left[MAXP + 2], right[MAXP + 2];
  double ndu[MAXP + 1][MAXP + 1];  // ndu[j][r]: basis of degree j (upper) and knot differences (lower)
  ndu[0][0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = u - t[s + 1 - j];
    right[j] = t[s + j] - u;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      ndu[j][r] = right[r + 1] + left[j - r];
      double tmp = ndu[j][r] != 0.0 ? ndu[r][j - 1] / ndu[j][r] : 0.0;
      ndu[r][j] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    ndu[j][j] = saved;
  }
  for (int r = 0; r <= p; ++r) val[r] = ndu[r][p];
  if (p == 0) {
    der[0] = 0.0;
    return;
  }
  // first derivative: p * (N_{r,p-1}/(t_{r+p}-t_r) - N_{r+1,p-1}/(t_{r+p+1}-t_{r+1}))
  for (int r = 0; r <= p; ++r) {
    double d = 0.0;
    if (r >= 1) {
      double den = ndu[p][r - 1];
      if (den != 0.0) d += ndu[r - 1][p - 1] / den;
    }
    if (r <= p - 1) {
      double den = ndu[p][r];
      if (den != 0.0) d -= ndu[r][p - 1] / den;
    }
    der[r] = p * d;
  }
}

struct Dir {
  int p = 0, n = 0, ne = 0, ng = 0;
  std::vector<double> knots;
  std::vector<int> span;       // knot index of each nonzero span (element)
  std::vector<double> tab;     // [e][g][a][2]
  std::vector<double> w;       // [e][g]
  std::vector<int> adj_first;  // first overlapping function of i (overlaps are contiguous)
  std::vector<int> adj_cnt;
  std::vector<int> adj_ptr;    // prefix over i
  std::vector<int> pair_elo, pair_ecnt;  // per 1D pair (indexed by adj_ptr[i] + b)
};

lam_status check_open_knots(int p, int nk, const double *k) {
  if (p < 1 || p > MAXP) return LAM_EUNSUP;
  if (!k || nk < 2 * p + 2) return LAM_EKNOT;
  for (int i = 0; i < nk; ++i)
    if (!std::isfinite(k[i])) return LAM_EKNOT;
  for (int i = 0; i + 1 < nk; ++i)
    if (!(k[i + 1] >= k[i])) return LAM_EKNOT;
  for (int i = 0; i <= p; ++i)
    if (k[i] != 0.0 || k[nk - 1 - i] != 1.0) return LAM_EKNOT;
  // a knot repeated more than p times would split the space (not open inside)
  for (int i = p + 1; i + p + 1 < nk; ++i) {
    int m = 1;
    while (i + m < nk - p - 1 && k[i + m] == k[i]) ++m;
    if (m > p) return LAM_EKNOT;
  }
  return LAM_OK;
}

void build_dir(Dir &d, int p, int nk, const double *k, int ng) {
  d.p = p;
  d.ng = ng;
  d.knots.assign(k, k + nk);
  d.n = nk - p - 1;
  for (int s = p; s < d.n; ++s)
    if (k[s + 1] > k[s]) d.span.push_back(s);
  d.ne = (int)d.span.size();
  double gx[MAXG], gw[MAXG];
  gauss_rule(ng, gx, gw);
  d.tab.assign((size_t)d.ne * ng * (p + 1) * 2, 0.0);
  d.w.assign((size_t)d.ne * ng, 0.0);
  for (int e = 0; e < d.ne; ++e) {
    int s = d.span[e];
    double a = k[s], b = k[s + 1], h = 0.5 * (b - a), c = 0.5 * (a + b);
    for (int g = 0; g < ng; ++g) {
      double val[MAXP + 1], der[MAXP + 1];
      basis_and_derivative(p, k, s, c + h * gx[g], val, der);
      for (int r = 0; r <= p; ++r) {
        d.tab[(((size_t)e * ng + g) * (p + 1) + r) * 2 + 0] = val[r];
        d.tab[(((size_t)e * ng + g) * (p + 1) + r) * 2 + 1] = der[r];
      }
      d.w[(size_t)e * ng + g] = gw[g] * h;
    }
  }
  // overlaps: i and j overlap iff some element carries both (its functions are span-p..span)
  d.adj_first.assign(d.n, 0);
  d.adj_cnt.assign(d.n, 0);
  for (int i = 0; i < d.n; ++i) {
    int lo = 1 << 30, hi = -1;
    for (int e = 0; e < d.ne; ++e) {
      int f = d.span[e] - p;
      if (i >= f && i <= f + p) {
        lo = std::min(lo, f);
        hi = std::max(hi, f + p);
      }
    }
    d.adj_first[i] = lo;
    d.adj_cnt[i] = hi - lo + 1;
  }
  d.adj_ptr.assign(d.n + 1, 0);
  for (int i = 0; i < d.n; ++i) d.adj_ptr[i + 1] = d.adj_ptr[i] + d.adj_cnt[i];
  d.pair_elo.assign(d.adj_ptr[d.n], 0);
  d.pair_ecnt.assign(d.adj_ptr[d.n], 0);
  for (int i = 0; i < d.n; ++i)
    for (int b = 0; b < d.adj_cnt[i]; ++b) {
      int j = d.adj_first[i] + b;
      int lo = -1, cnt = 0;
      for (int e = 0; e < d.ne; ++e) {
        int f = d.span[e] - p;
        if (i >= f && i <= f + p && j >= f && j <= f + p) {
          if (lo < 0) lo = e;
          ++cnt;
        }
      }
      d.pair_elo[d.adj_ptr[i] + b] = lo;
      d.pair_ecnt[d.adj_ptr[i] + b] = cnt;
    }
}

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct Builder {
  lam::Layout &L;
  int64_t cur = 0;
  explicit Builder(lam::Layout &l) : L(l) {}
  lam::Region take(int64_t bytes) {
    lam::Region r;
    r.off = cur;
    r.bytes = bytes;
    cur = align256(cur + std::max<int64_t>(bytes, 1));
    return r;
  }
};

template <class T>
void put(std::vector<uint8_t> &img, const lam::Region &r, const std::vector<T> &v) {
  if (!v.empty()) std::memcpy(img.data() + r.off, v.data(), v.size() * sizeof(T));
}

}  // namespace

namespace lam {

// min_nsc: smallest number of set slots of the register-mode scatter (the
// batched path compiles one slot count for every laminate).
lam_status plan_create(const lam_laminate_desc *d, const lam_tuning *tune, int min_nsc, lam_plan **out,
                       const lam_shell *shell) {
  if (!d || !out) return LAM_EINVAL;
  *out = nullptr;
  lam_status st;
  if ((st = check_open_knots(d->p1, d->nk1, d->k1)) != LAM_OK) return st;
  if ((st = check_open_knots(d->p2, d->nk2, d->k2)) != LAM_OK) return st;
  if ((st = check_open_knots(d->q, d->nk3, d->k3)) != LAM_OK) return st;
  if (d->set_mode < LAM_SETS_BUCKET || d->set_mode > LAM_SETS_PLY) return LAM_EINVAL;
  if (d->n_ply < 1 || d->n_ply > 4096 || !d->iface || !d->ply_mat) return LAM_EPLY;
  if (d->n_mat < 1 || d->n_mat > 64) return LAM_EINVAL;
  if (d->set_mode == LAM_SETS_BUCKET && !d->ply_theta) return LAM_EINVAL;
  if (d->iface[0] != 0.0 || d->iface[d->n_ply] != 1.0) return LAM_EPLY;
  for (int l = 0; l < d->n_ply; ++l) {
    if (!std::isfinite(d->iface[l + 1]) || !(d->iface[l + 1] > d->iface[l])) return LAM_EPLY;
    if (d->ply_mat[l] < 0 || d->ply_mat[l] >= d->n_mat) return LAM_EPLY;
    if (d->set_mode == LAM_SETS_BUCKET && !std::isfinite(d->ply_theta[l])) return LAM_EMAT;
  }
  int ng1 = d->ng1 ? d->ng1 : d->p1 + 1, ng2 = d->ng2 ? d->ng2 : d->p2 + 1, ngz = d->ngz ? d->ngz : d->q + 1;
  if (ng1 < 1 || ng1 > MAXG || ng2 < 1 || ng2 > MAXG || ngz < 1 || ngz > MAXG) return LAM_EUNSUP;
  if (shell) {
    if (!shell->ctrl || (shell->mat_field != 0 && shell->mat_field != 1)) return LAM_EINVAL;
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(shell->a[a])) return LAM_EMAT;
    // a material field is assembled per set from its own 2D integrals (no
    // harmonic decomposition of a field)
    if (shell->mat_field && d->set_mode != LAM_SETS_BUCKET && d->set_mode != LAM_SETS_PLY) return LAM_EUNSUP;
  }
  double cof[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, det = 1.0;
  if (!shell) {
    const double *J = d->jac;
    for (int a = 0; a < 9; ++a)
      if (!std::isfinite(J[a])) return LAM_EMAT;
    double c9[9] = {J[4] * J[8] - J[5] * J[7], -(J[3] * J[8] - J[5] * J[6]), J[3] * J[7] - J[4] * J[6],
                    -(J[1] * J[8] - J[2] * J[7]), J[0] * J[8] - J[2] * J[6], -(J[0] * J[7] - J[1] * J[6]),
                    J[1] * J[5] - J[2] * J[4], -(J[0] * J[5] - J[2] * J[3]), J[0] * J[4] - J[1] * J[3]};
    std::memcpy(cof, c9, sizeof(cof));
    det = J[0] * cof[0] + J[1] * cof[1] + J[2] * cof[2];
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return LAM_EMAT;
  }

  lam_plan *P = new (std::nothrow) lam_plan();
  if (!P) return LAM_EINVAL;
  // DF^{-1} = cof^T / det, so DF^{-T} = cof / det (a shell's vary per point: gtab)
  for (int a = 0; a < 9; ++a) P->jit[a] = cof[a] / det;
  P->detj = std::fabs(det);
  P->shell = shell ? 1 : 0;
  P->mat_field = shell ? shell->mat_field : 0;
  P->p1 = d->p1;
  P->p2 = d->p2;
  P->q = d->q;
  P->ng1 = ng1;
  P->ng2 = ng2;
  P->ngz = ngz;
  P->n_ply = d->n_ply;
  P->n_mat = d->n_mat;
  // one set per ply is bucket grouping with every ply its own bucket
  P->set_mode = d->set_mode == LAM_SETS_PLY ? LAM_SETS_BUCKET : d->set_mode;

  Dir d1, d2, dz;
  build_dir(d1, d->p1, d->nk1, d->k1, ng1);
  build_dir(d2, d->p2, d->nk2, d->k2, ng2);
  P->n1 = d1.n;
  P->n2 = d2.n;
  P->ne1 = d1.ne;
  P->ne2 = d2.ne;
  P->ns = d1.n * d2.n;

  // ---- curved shell: basis (B-spline products or NURBS quotients) and the
  // map gradient DF = [dS/dxi1 | dS/dxi2 | a] at every in-plane Gauss point
  std::vector<double> gtab, rtab;
  if (shell) {
    const int P1 = d->p1 + 1, P2 = d->p2 + 1, nb = P1 * P2, ngp = ng1 * ng2;
    for (int i = 0; i < 3 * P->ns; ++i)
      if (!std::isfinite(shell->ctrl[i])) {
        delete P;
        return LAM_EMAT;
      }
    if (shell->weights)
      for (int i = 0; i < P->ns; ++i)
        if (!std::isfinite(shell->weights[i]) || !(shell->weights[i] > 0.0)) {
          delete P;
          return LAM_EMAT;
        }
    gtab.assign((size_t)d1.ne * d2.ne * ngp * 10, 0.0);
    rtab.assign((size_t)d1.ne * d2.ne * ngp * nb * 3, 0.0);
    for (int e2 = 0; e2 < d2.ne; ++e2)
      for (int e1 = 0; e1 < d1.ne; ++e1) {
        const int e = e1 + d1.ne * e2, f1 = d1.span[e1] - d->p1, f2 = d2.span[e2] - d->p2;
        for (int g2 = 0; g2 < ng2; ++g2)
          for (int g1 = 0; g1 < ng1; ++g1) {
            const int g = g1 + ng1 * g2;
            double *rb = &rtab[((size_t)e * ngp + g) * nb * 3];
            const double *t1 = &d1.tab[((size_t)e1 * ng1 + g1) * P1 * 2];
            const double *t2 = &d2.tab[((size_t)e2 * ng2 + g2) * P2 * 2];
            double W = 0.0, W1 = 0.0, W2 = 0.0;
            for (int b2 = 0; b2 < P2; ++b2)
              for (int b1 = 0; b1 < P1; ++b1) {
                const int b = b2 * P1 + b1;
                const double w = shell->weights ? shell->weights[(f2 + b2) * P->n1 + f1 + b1] : 1.0;
                rb[3 * b + 0] = w * t1[2 * b1] * t2[2 * b2];
                rb[3 * b + 1] = w * t1[2 * b1 + 1] * t2[2 * b2];
                rb[3 * b + 2] = w * t1[2 * b1] * t2[2 * b2 + 1];
                W += rb[3 * b];
                W1 += rb[3 * b + 1];
                W2 += rb[3 * b + 2];
              }
            if (shell->weights)  // R = w N / W; dR = (w dN - R dW) / W
              for (int b = 0; b < nb; ++b) {
                const double r = rb[3 * b] / W;
                rb[3 * b + 1] = (rb[3 * b + 1] - r * W1) / W;
                rb[3 * b + 2] = (rb[3 * b + 2] - r * W2) / W;
                rb[3 * b] = r;
              }
            double Jm[9] = {0, 0, shell->a[0], 0, 0, shell->a[1], 0, 0, shell->a[2]};
            for (int b2 = 0; b2 < P2; ++b2)
              for (int b1 = 0; b1 < P1; ++b1) {
                const int b = b2 * P1 + b1;
                const double *X = shell->ctrl + 3 * (size_t)((f2 + b2) * P->n1 + f1 + b1);
                for (int r = 0; r < 3; ++r) {
                  Jm[3 * r + 0] += rb[3 * b + 1] * X[r];
                  Jm[3 * r + 1] += rb[3 * b + 2] * X[r];
                }
              }
            const double c9[9] = {Jm[4] * Jm[8] - Jm[5] * Jm[7], -(Jm[3] * Jm[8] - Jm[5] * Jm[6]),
                                  Jm[3] * Jm[7] - Jm[4] * Jm[6], -(Jm[1] * Jm[8] - Jm[2] * Jm[7]),
                                  Jm[0] * Jm[8] - Jm[2] * Jm[6], -(Jm[0] * Jm[7] - Jm[1] * Jm[6]),
                                  Jm[1] * Jm[5] - Jm[2] * Jm[4], -(Jm[0] * Jm[5] - Jm[2] * Jm[3]),
                                  Jm[0] * Jm[4] - Jm[1] * Jm[3]};
            const double dt = Jm[0] * c9[0] + Jm[1] * c9[1] + Jm[2] * c9[2];
            if (!(std::fabs(dt) > 0.0) || !std::isfinite(dt)) {
              delete P;
              return LAM_EMAT;
            }
            double *gb = &gtab[((size_t)e * ngp + g) * 10];
            for (int a = 0; a < 9; ++a) gb[a] = c9[a] / dt;
            gb[9] = d1.w[(size_t)e1 * ng1 + g1] * d2.w[(size_t)e2 * ng2 + g2] * std::fabs(dt);
          }
      }
  }

  // ---- thickness: cells = (ply, nonzero knot span) intersections, bottom to top
  Dir zs;
  zs.p = d->q;
  zs.knots.assign(d->k3, d->k3 + d->nk3);
  zs.n = d->nk3 - d->q - 1;
  for (int s = d->q; s < zs.n; ++s)
    if (d->k3[s + 1] > d->k3[s]) zs.span.push_back(s);
  P->nt = zs.n;
  std::vector<int> zfirst, zply;
  std::vector<double> ztab, zw;
  double gx[MAXG], gw[MAXG];
  gauss_rule(ngz, gx, gw);
  for (int l = 0; l < d->n_ply; ++l)
    for (int s : zs.span) {
      double a = std::max(d->iface[l], d->k3[s]), b = std::min(d->iface[l + 1], d->k3[s + 1]);
      if (!(b > a)) continue;
      zfirst.push_back(s - d->q);
      zply.push_back(l);
      double h = 0.5 * (b - a), c = 0.5 * (a + b);
      for (int g = 0; g < ngz; ++g) {
        double val[MAXP + 1], der[MAXP + 1];
        basis_and_derivative(d->q, d->k3, s, c + h * gx[g], val, der);
        for (int r = 0; r <= d->q; ++r) {
          ztab.push_back(val[r]);
          ztab.push_back(der[r]);
        }
        zw.push_back(gw[g] * h);
      }
    }
  P->nzc = (int)zfirst.size();
  // thickness overlap (contiguous ranges) and the cells shared by each pair
  std::vector<int> zrow(P->nt + 1, 0), zcol, zkrow, zcptr(1, 0), zcell;
  for (int it = 0; it < P->nt; ++it) {
    int lo = 1 << 30, hi = -1;
    for (int s : zs.span) {
      int f = s - d->q;
      if (it >= f && it <= f + d->q) {
        lo = std::min(lo, f);
        hi = std::max(hi, f + d->q);
      }
    }
    for (int jt = lo; jt <= hi; ++jt) {
      zcol.push_back(jt);
      zkrow.push_back(it);
      for (int c = 0; c < P->nzc; ++c) {
        int f = zfirst[c];
        if (it >= f && it <= f + d->q && jt >= f && jt <= f + d->q) zcell.push_back(c);
      }
      zcptr.push_back((int)zcell.size());
    }
    zrow[it + 1] = (int)zcol.size();
  }
  P->nnzz = (int64_t)zcol.size();

  // ---- in-plane pattern: row is = i1 + n1*i2, columns (j2, j1) ascending
  std::vector<int> srow(P->ns + 1, 0);
  for (int i2 = 0; i2 < d2.n; ++i2)
    for (int i1 = 0; i1 < d1.n; ++i1) {
      int is = i1 + d1.n * i2;
      srow[is + 1] = d1.adj_cnt[i1] * d2.adj_cnt[i2];
    }
  for (int is = 0; is < P->ns; ++is) srow[is + 1] += srow[is];
  P->nnz2 = srow[P->ns];
  P->nnz1 = d1.adj_ptr[d1.n];
  std::vector<int> krow(P->nnz2), kcol(P->nnz2), kp1(P->nnz2), kp2(P->nnz2);
  for (int i2 = 0; i2 < d2.n; ++i2)
    for (int i1 = 0; i1 < d1.n; ++i1) {
      int is = i1 + d1.n * i2, k = srow[is];
      for (int b2 = 0; b2 < d2.adj_cnt[i2]; ++b2)
        for (int b1 = 0; b1 < d1.adj_cnt[i1]; ++b1, ++k) {
          krow[k] = is;
          kcol[k] = (d1.adj_first[i1] + b1) + d1.n * (d2.adj_first[i2] + b2);
          kp1[k] = d1.adj_ptr[i1] + b1;
          kp2[k] = d2.adj_ptr[i2] + b2;
        }
    }
  P->nnz = 9 * P->nnz2 * P->nnzz;
  P->nrows = 3 * (int64_t)P->ns * P->nt;
  if ((int64_t)3 * P->ns * P->nt >= (int64_t(1) << 31) || P->nnz2 >= (int64_t(1) << 31) ||
      P->nnz >= (int64_t(1) << 62)) {
    delete P;
    return LAM_EUNSUP;
  }

  // ---- sets
  std::vector<int> set_mat, set_aux, ply_set(d->n_ply, -1);
  if (d->set_mode == LAM_SETS_PLY) {
    for (int l = 0; l < d->n_ply; ++l) {
      ply_set[l] = (int)set_mat.size();
      set_mat.push_back(d->ply_mat[l]);
      set_aux.push_back(l);
    }
    P->n_harm = 0;
  } else if (d->set_mode == LAM_SETS_BUCKET) {
    std::map<std::pair<int, uint64_t>, int> key;
    for (int l = 0; l < d->n_ply; ++l) {
      uint64_t bits;
      double th = d->ply_theta[l] == 0.0 ? 0.0 : d->ply_theta[l];  // -0 == +0
      std::memcpy(&bits, &th, 8);
      auto k = std::make_pair((int)d->ply_mat[l], bits);
      auto itk = key.find(k);
      if (itk == key.end()) {
        int s = (int)set_mat.size();
        key[k] = s;
        set_mat.push_back(d->ply_mat[l]);
        set_aux.push_back(l);  // representative ply: its runtime angle defines the set
        ply_set[l] = s;
      } else {
        ply_set[l] = itk->second;
      }
    }
    P->n_harm = 0;
  } else {
    P->n_harm = d->set_mode == LAM_SETS_HARMONIC5 ? 5 : 9;
    std::vector<int> used(d->n_mat, 0);
    for (int l = 0; l < d->n_ply; ++l) used[d->ply_mat[l]] = 1;
    std::vector<int> first_set(d->n_mat, -1);
    for (int m = 0; m < d->n_mat; ++m) {
      if (!used[m]) continue;
      first_set[m] = (int)set_mat.size();
      for (int h = 0; h < P->n_harm; ++h) {
        set_mat.push_back(m);
        set_aux.push_back(h);
      }
    }
    for (int l = 0; l < d->n_ply; ++l) ply_set[l] = first_set[d->ply_mat[l]];  // first harmonic of its material
  }
  P->n_sets = (int)set_mat.size();
  // Harmonic sets are evaluated per ply when at most two plies touch any
  // thickness row (layerwise spaces): the scatter's sets are then the plies,
  // each ply's tensor the sum of its material's harmonics with the ply's
  // weights, which keeps two set slots instead of n_harm per material.
  if (P->set_mode != LAM_SETS_BUCKET) {
    int most = 0;
    for (int it = 0; it < P->nt; ++it) {
      std::vector<int> pl;
      for (int c = 0; c < P->nzc; ++c)
        if (it >= zfirst[c] && it <= zfirst[c] + d->q) pl.push_back(zply[c]);
      std::sort(pl.begin(), pl.end());
      most = std::max(most, (int)(std::unique(pl.begin(), pl.end()) - pl.begin()));
    }
    P->harm_ply = most <= 2 ? 1 : 0;
  }
  // sets active on each thickness row: those of plies with a cell in the row's support
  std::vector<int> zaptr(P->nt + 1, 0), zaset;
  int maxact = 0;
  for (int it = 0; it < P->nt; ++it) {
    std::vector<int> act;
    for (int c = 0; c < P->nzc; ++c) {
      if (it < zfirst[c] || it > zfirst[c] + d->q) continue;
      int l = zply[c];
      if (P->set_mode == LAM_SETS_BUCKET) {
        act.push_back(ply_set[l]);
      } else if (P->harm_ply) {
        act.push_back(l);
      } else {
        for (int h = 0; h < P->n_harm; ++h) act.push_back(ply_set[l] + h);
      }
    }
    std::sort(act.begin(), act.end());
    act.erase(std::unique(act.begin(), act.end()), act.end());
    maxact = std::max(maxact, (int)act.size());
    zaset.insert(zaset.end(), act.begin(), act.end());
    zaptr[it + 1] = (int)zaset.size();
  }
  P->maxact = std::max(maxact, 1);

  // ---- Kronecker scatter tiles and chunks.
  // A tile is a run of whole in-plane rows (at most 85 in-plane nonzeros, one
  // thread per (nonzero, component) slot), so that for every thickness row one
  // block writes one contiguous range of the CSR values and no cache line is
  // shared between blocks except at the two ends of the range.  A chunk is a
  // run of thickness rows whose active sets fit the block's set slots.
  //  - register mode (every row needs at most 8 sets): each thread keeps P of
  //    the chunk's sets for its slot in registers (kron_nsc slots: 1, 2, 4 or 8)
  //    and reads the slot-dense coefficients Qd with scalar loads;
  //  - LDS mode (more sets per row): the tile's P of the chunk's sets and the
  //    chunk's coefficients Qc are staged in LDS.
  const int64_t per_k = 36 * (int64_t)sizeof(double);  // P bytes per in-plane nonzero and set
  int max_ls = 0;
  for (int is = 0; is < P->ns; ++is) max_ls = std::max(max_ls, srow[is + 1] - srow[is]);
  // whole rows of the typical (interior) length fill a 256-thread block best
  int tk_target = max_ls > 0 ? max_ls * std::max(1, 85 / max_ls) : 85;
  if (tune && tune->tile_k > 0) tk_target = std::min(85, tune->tile_k);
  tk_target = std::max(tk_target, max_ls);
  if (tk_target > 85) {
    delete P;
    return LAM_EUNSUP;
  }
  int nsc_cap = 2;  // fewer slots keep more waves resident; chunks reload P from cache
  if (tune && tune->set_slots > 0) nsc_cap = tune->set_slots;
  // material fields: P of every set is integrated over the plane with the
  // field inside and stored; the register-mode scatter loads it per chunk
  // (one or two slots), the LDS-mode scatter stages it
  const bool reg_mode = P->maxact <= (P->mat_field ? 2 : 8);
  if (P->mat_field) nsc_cap = 2;
  int sc, tkmax = tk_target;
  int64_t qbudget = 8 * 1024, lds_budget = 80 * 1024;
  if (tune && tune->lds_kib > 0) lds_budget = std::max<int64_t>(16 * 1024, (int64_t)tune->lds_kib * 1024);
  if (reg_mode) {
    int want = std::max(std::max(P->maxact, std::min(P->n_sets, nsc_cap)), min_nsc);
    sc = want <= 1 ? 1 : want <= 2 ? 2 : want <= 4 ? 4 : 8;
    P->kron_nsc = sc;
  } else {
    // largest tile whose P of every set and coefficients fit; else as many
    // sets as fit next to a one-row tile; else P is read from memory
    sc = 0;
    for (int tk = tk_target; tk >= max_ls; --tk)
      if (per_k * tk * P->n_sets + qbudget <= lds_budget) {
        tkmax = tk;
        sc = P->n_sets;
        break;
      }
    if (sc == 0) {
      tkmax = max_ls;
      sc = (int)std::min<int64_t>(P->n_sets, (lds_budget - qbudget) / (per_k * tkmax));
    }
    if (sc < P->maxact) {
      tkmax = tk_target;
      sc = 0;
    }
    P->kron_nsc = 0;
  }
  const bool lds_sets = !reg_mode && sc > 0;
  std::vector<int> tiles(1, 0);
  int tk_real = 0;
  for (int is = 0; is < P->ns; ++is) {
    int cur = srow[is + 1] - tiles.back();
    if (cur > tkmax) {
      tk_real = std::max(tk_real, srow[is] - tiles.back());
      tiles.push_back(srow[is]);
    }
  }
  tk_real = std::max<int>(tk_real, (int)P->nnz2 - tiles.back());
  tiles.push_back((int)P->nnz2);
  P->n_tiles = (int)tiles.size() - 1;
  P->tile_k = tk_real;
  P->kron_threads = std::min(256, 64 * ((3 * tk_real + 63) / 64));
  // chunks of consecutive thickness rows: the union of their active sets fits
  // sc slots (register mode, LDS-set mode) and, in LDS mode, their
  // coefficients fit qbudget bytes
  const int64_t q_per_zk = 4 * (int64_t)sizeof(double) * P->maxact;
  std::vector<int> chunk_ptr(1, 0), chunk_sptr(1, 0), chunk_set, zaslot(zaset.size(), 0), zchunk(P->nt, 0);
  {
    std::vector<int> cur;
    int start = 0;
    int64_t qbytes = 0;
    const bool by_sets = reg_mode || lds_sets;
    std::vector<int> prev;  // the previous chunk's sets, in slot order
    auto flush = [&](int end) {
      // slot order: a set the previous chunk also had keeps its slot where it
      // fits, so that the scatter recomputes P only for the slots that change
      std::sort(cur.begin(), cur.end());
      std::vector<int> ord(cur.size(), -1);
      for (size_t w = 0; w < prev.size() && w < ord.size(); ++w)
        if (std::binary_search(cur.begin(), cur.end(), prev[w])) ord[w] = prev[w];
      for (int sset : cur)
        if (std::find(ord.begin(), ord.end(), sset) == ord.end()) *std::find(ord.begin(), ord.end(), -1) = sset;
      cur = ord;
      prev = ord;
      for (int it = start; it < end; ++it) {
        zchunk[it] = (int)chunk_ptr.size() - 1;
        for (int j = zaptr[it]; j < zaptr[it + 1]; ++j)
          zaslot[j] = by_sets ? (int)(std::find(cur.begin(), cur.end(), zaset[j]) - cur.begin()) : 0;
      }
      chunk_set.insert(chunk_set.end(), cur.begin(), cur.end());
      chunk_sptr.push_back((int)chunk_set.size());
      chunk_ptr.push_back(end);
      cur.clear();
      start = end;
      qbytes = 0;
    };
    for (int it = 0; it < P->nt; ++it) {
      int64_t qrow = q_per_zk * (zrow[it + 1] - zrow[it]);
      std::vector<int> uni = cur;
      if (by_sets)
        for (int j = zaptr[it]; j < zaptr[it + 1]; ++j)
          if (std::find(uni.begin(), uni.end(), zaset[j]) == uni.end()) uni.push_back(zaset[j]);
      bool over = by_sets && (int)uni.size() > sc;
      if (!reg_mode) over = over || qbytes + qrow > qbudget;
      if (it > start && over) {
        flush(it);
        uni.clear();
        if (by_sets) uni.assign(zaset.begin() + zaptr[it], zaset.begin() + zaptr[it + 1]);
      }
      cur = uni;
      qbytes += qrow;
    }
    flush(P->nt);
  }
  // enough blocks to keep every compute unit busy through the tail: split
  // chunks into pieces of at most max_rows rows; a piece keeps its chunk's
  // set list (and so the slots of zaslot)
  int64_t target_blocks = 6144;
  if (tune && tune->target_blocks > 0) target_blocks = tune->target_blocks;
  const int64_t per_tile = (target_blocks + P->n_tiles - 1) / P->n_tiles;
  int max_rows = (int)std::max<int64_t>(1, (P->nt + per_tile - 1) / per_tile);
  // with enough tiles to fill the chip, a piece keeps at least 8 rows (or the
  // whole thickness): each block pays its prologue once for its rows
  if (P->n_tiles >= 1024) max_rows = std::max(max_rows, std::min(P->nt, 8));
  {
    std::vector<int> cp(1, 0), csp(1, 0), cs;
    for (size_t c = 0; c + 1 < chunk_ptr.size(); ++c) {
      const int a = chunk_ptr[c], b = chunk_ptr[c + 1];
      const int pieces = (b - a + max_rows - 1) / max_rows;
      for (int q = 0; q < pieces; ++q) {
        const int e = a + (int)((int64_t)(b - a) * (q + 1) / pieces);
        for (int it = cp.back(); it < e; ++it) zchunk[it] = (int)cp.size() - 1;
        cp.push_back(e);
        cs.insert(cs.end(), chunk_set.begin() + chunk_sptr[c], chunk_set.begin() + chunk_sptr[c + 1]);
        csp.push_back((int)cs.size());
      }
    }
    chunk_ptr.swap(cp);
    chunk_sptr.swap(csp);
    chunk_set.swap(cs);
  }
  P->n_chunks = (int)chunk_ptr.size() - 1;
  P->chunk_sets = lds_sets ? sc : 0;
  // groups: runs of consecutive chunks that one register-mode block walks in
  // order after staging, once, the coefficients of all their thickness rows and
  // the bracket coefficients of all their sets; together at most max_rows
  // thickness rows, kGroupSets distinct sets and kGroupQBytes of coefficients.
  // Short chunks (a set change at every ply) then share the block's in-plane
  // moments, and the row loop of a block never waits on a load.  LDS mode and
  // four or eight slots keep one chunk per group.  chunk_lset: each chunk
  // slot's index in its group's set list.
  constexpr int kGroupSets = 16;
  constexpr int64_t kGroupQBytes = 4 * 1024;
  std::vector<int> group_ptr(1, 0), group_sptr(1, 0), group_set, chunk_lset(chunk_set.size(), 0);
  int max_group_zk = 0, max_group_sets = 0;
  {
    std::vector<int> gsets;
    int rows = 0, gzk = 0;
    auto flush = [&](int end) {
      for (int c = group_ptr.back(); c < end; ++c)
        for (int j = chunk_sptr[c]; j < chunk_sptr[c + 1]; ++j)
          chunk_lset[j] = (int)(std::find(gsets.begin(), gsets.end(), chunk_set[j]) - gsets.begin());
      group_set.insert(group_set.end(), gsets.begin(), gsets.end());
      group_sptr.push_back((int)group_set.size());
      group_ptr.push_back(end);
      max_group_zk = std::max(max_group_zk, gzk);
      max_group_sets = std::max(max_group_sets, (int)gsets.size());
      gsets.clear();
      rows = gzk = 0;
    };
    const int64_t q_per_zk_reg = 4 * (int64_t)sizeof(double) * std::max(P->kron_nsc, 1);
    for (int c = 0; c < P->n_chunks; ++c) {
      const int r = chunk_ptr[c + 1] - chunk_ptr[c], zk = zrow[chunk_ptr[c + 1]] - zrow[chunk_ptr[c]];
      int fresh = 0;
      for (int j = chunk_sptr[c]; j < chunk_sptr[c + 1]; ++j)
        fresh += std::find(gsets.begin(), gsets.end(), chunk_set[j]) == gsets.end();
      if (c > group_ptr.back() && (!reg_mode || P->kron_nsc > 2 || rows + r > max_rows || (int)gsets.size() + fresh > kGroupSets ||
                                   q_per_zk_reg * (gzk + zk) > kGroupQBytes))
        flush(c);
      for (int j = chunk_sptr[c]; j < chunk_sptr[c + 1]; ++j)
        if (std::find(gsets.begin(), gsets.end(), chunk_set[j]) == gsets.end()) gsets.push_back(chunk_set[j]);
      rows += r;
      gzk += zk;
    }
    flush(P->n_chunks);
  }
  P->n_groups = (int)group_ptr.size() - 1;
  int max_chunk_zk = 0;
  for (int c = 0; c < P->n_chunks; ++c)
    max_chunk_zk = std::max(max_chunk_zk, zrow[chunk_ptr[c + 1]] - zrow[chunk_ptr[c]]);
  if (reg_mode) {
    // the group's coefficients, then the bracket coefficients of its sets and
    // one zero block (one or two slots) or of each slot (four or eight)
    P->kron_lds_q = 4 * (int64_t)sizeof(double) * P->kron_nsc * max_group_zk;
    P->kron_lds_p = 81 * (int64_t)sizeof(double) * std::max(max_group_sets + 1, P->kron_nsc);
    P->kron_lds = P->kron_lds_q + P->kron_lds_p;
    if (P->kron_lds > 64 * 1024) {
      delete P;
      return LAM_EUNSUP;
    }
  } else {
    P->kron_lds_q = 4 * (int64_t)sizeof(double) * P->maxact * max_chunk_zk;
    P->kron_lds_p = per_k * tkmax * P->chunk_sets;
    P->kron_lds = P->kron_lds_q + P->kron_lds_p;
    if (P->kron_lds > 160 * 1024) {
      delete P;
      return LAM_EUNSUP;  // one thickness row's coefficients exceed the LDS of a compute unit
    }
  }

  // ---- standard assembly: 1D overlap ranges, thickness spans and their cells
  std::vector<int> a1f(d1.adj_first), a1c(d1.adj_cnt), a2f(d2.adj_first), a2c(d2.adj_cnt);
  std::vector<int> zs_first, zs_cptr(1, 0), zs_cell;
  for (int s3 : zs.span) {
    zs_first.push_back(s3 - d->q);
    for (int c = 0; c < P->nzc; ++c)
      if (zfirst[c] == s3 - d->q) zs_cell.push_back(c);
    zs_cptr.push_back((int)zs_cell.size());
  }
  P->nzs = (int)zs.span.size();
  {
    int mx = 0;
    for (int z = 0; z < P->nzs; ++z) mx = std::max(mx, zs_cptr[z + 1] - zs_cptr[z]);
    P->max_span_cells = mx;
  }

  // ---- adjoint: every thickness pair touches at most two plies, kept in
  // accumulator slot (ply & 1); a ply's accumulators are reduced after the last
  // thickness row that touches it
  std::vector<int> rowply(2 * (size_t)P->nt, -1), rowfin(P->nt, 0), last_row(d->n_ply, -1);
  P->adj_ok = 1;
  for (int it = 0; it < P->nt; ++it)
    for (int zk = zrow[it]; zk < zrow[it + 1]; ++zk)
      for (int ci = zcptr[zk]; ci < zcptr[zk + 1]; ++ci) {
        const int l = zply[zcell[ci]], slot = l & 1;
        if (rowply[2 * it + slot] >= 0 && rowply[2 * it + slot] != l) P->adj_ok = 0;
        rowply[2 * it + slot] = l;
        last_row[l] = std::max(last_row[l], it);
      }
  std::vector<int> first_row(d->n_ply, -1);
  for (int it = P->nt - 1; it >= 0; --it)
    for (int sl = 0; sl < 2; ++sl)
      if (rowply[2 * it + sl] >= 0) first_row[rowply[2 * it + sl]] = it;
  for (int l = 0; l < d->n_ply; ++l) {
    if (last_row[l] < 0) continue;
    rowfin[last_row[l]] |= 1 << (l & 1);
    // a ply whose slot another ply took on every row it touches: unsupported
    if (first_row[l] < 0) {
      P->adj_ok = 0;
      continue;
    }
    // while ply l accumulates, no other ply may use its slot
    for (int it = first_row[l]; it <= last_row[l]; ++it) {
      const int o = rowply[2 * it + (l & 1)];
      if (o >= 0 && o != l) P->adj_ok = 0;
    }
  }

  if (P->mat_field) P->adj_ok = 0;  // the adjoint's per-ply 6x6 gradient does not describe a field
  std::vector<int> plymat(d->ply_mat, d->ply_mat + d->n_ply);

  // ---- layout
  lam::Layout &L = P->L;
  Builder B(L);
  L.tab1 = B.take(sizeof(double) * d1.tab.size());
  L.w1 = B.take(sizeof(double) * d1.w.size());
  L.tab2 = B.take(sizeof(double) * d2.tab.size());
  L.w2 = B.take(sizeof(double) * d2.w.size());
  L.e1first = B.take(sizeof(int) * d1.ne);
  L.e2first = B.take(sizeof(int) * d2.ne);
  L.pe1 = B.take(sizeof(int) * 2 * d1.pair_elo.size());
  L.pe2 = B.take(sizeof(int) * 2 * d2.pair_elo.size());
  L.srow = B.take(sizeof(int) * srow.size());
  L.krow = B.take(sizeof(int) * krow.size());
  L.kcol = B.take(sizeof(int) * kcol.size());
  L.kp1 = B.take(sizeof(int) * kp1.size());
  L.kp2 = B.take(sizeof(int) * kp2.size());
  L.zfirst = B.take(sizeof(int) * zfirst.size());
  L.zply = B.take(sizeof(int) * zply.size());
  L.ztab = B.take(sizeof(double) * ztab.size());
  L.zw = B.take(sizeof(double) * zw.size());
  L.zrow = B.take(sizeof(int) * zrow.size());
  L.zcol = B.take(sizeof(int) * zcol.size());
  L.zkrow = B.take(sizeof(int) * zkrow.size());
  L.zcptr = B.take(sizeof(int) * zcptr.size());
  L.zcell = B.take(sizeof(int) * zcell.size());
  L.zaptr = B.take(sizeof(int) * zaptr.size());
  L.zaset = B.take(sizeof(int) * zaset.size());
  L.a1f = B.take(sizeof(int) * a1f.size());
  L.a1c = B.take(sizeof(int) * a1c.size());
  L.a2f = B.take(sizeof(int) * a2f.size());
  L.a2c = B.take(sizeof(int) * a2c.size());
  L.zs_first = B.take(sizeof(int) * zs_first.size());
  L.zs_cptr = B.take(sizeof(int) * zs_cptr.size());
  L.zs_cell = B.take(sizeof(int) * zs_cell.size());
  L.rowply = B.take(sizeof(int) * rowply.size());
  L.rowfin = B.take(sizeof(int) * rowfin.size());
  L.set_mat = B.take(sizeof(int) * set_mat.size());
  L.set_aux = B.take(sizeof(int) * set_aux.size());
  L.ply_mat = B.take(sizeof(int) * plymat.size());
  L.ply_set = B.take(sizeof(int) * ply_set.size());
  L.tiles = B.take(sizeof(int) * tiles.size());
  L.zchunk = B.take(sizeof(int) * zchunk.size());
  L.chunk_ptr = B.take(sizeof(int) * chunk_ptr.size());
  L.group_ptr = B.take(sizeof(int) * group_ptr.size());
  L.group_sptr = B.take(sizeof(int) * group_sptr.size());
  L.group_set = B.take(sizeof(int) * group_set.size());
  L.chunk_lset = B.take(sizeof(int) * chunk_lset.size());
  L.chunk_sptr = B.take(sizeof(int) * chunk_sptr.size());
  L.chunk_set = B.take(sizeof(int) * chunk_set.size());
  L.zaslot = B.take(sizeof(int) * zaslot.size());
  L.gtab = B.take(sizeof(double) * gtab.size());
  L.rtab = B.take(sizeof(double) * rtab.size());
  L.status = B.take(sizeof(int) * lam::N_STATUS);
  L.const_bytes = B.cur;
  L.D = B.take(sizeof(double) * 36 * P->n_sets);
  L.Ec = B.take(sizeof(double) * 81 * P->n_sets);
  // P of every set is stored only by the LDS-mode scatter; the register mode
  // contracts it from the moments M
  L.P = B.take(P->kron_nsc > 0 && !P->mat_field ? 0 : sizeof(double) * 36 * (int64_t)P->n_sets * P->nnz2);
  L.Qc = B.take(sizeof(double) * 4 * (int64_t)std::max(P->maxact, P->kron_nsc) * P->nnzz);
  L.M = B.take(sizeof(double) * 36 * ((P->nnz2 + 63) / 64 * 64));  // blocks of 64 nonzeros (m_index)
  L.Eply = B.take(sizeof(double) * 81 * P->n_ply);
  L.Ectl = B.take(P->mat_field ? sizeof(double) * 81 * (int64_t)P->n_sets * P->ns : 0);
  L.Epts = B.take(P->mat_field ? sizeof(double) * 81 * (int64_t)P->n_sets * P->ne1 * P->ne2 * ng1 * ng2 : 0);
  L.fwd_end = B.cur;  // scratch of the fast assembly ends here
  // adjoint scratch: per-ply 1D operators by slot (padded per thickness row), per (ply, tile) partial sums,
  // per-ply totals and dL/dD_l
  L.Qp = B.take(sizeof(double) * 8 * std::max<int64_t>(P->nnzz, (int64_t)P->nt * (2 * P->q + 1)));
  L.adj_part = B.take(sizeof(double) * 81 * (int64_t)P->n_tiles * P->n_ply);
  L.adj_y = B.take(sizeof(double) * 81 * P->n_ply);
  L.adj_cm = B.take(sizeof(double) * 36 * P->n_ply);
  L.total = B.cur;

  P->image.assign(L.const_bytes, 0);
  auto &img = P->image;
  put(img, L.tab1, d1.tab);
  put(img, L.w1, d1.w);
  put(img, L.tab2, d2.tab);
  put(img, L.w2, d2.w);
  {
    std::vector<int> f(d1.ne);
    for (int e = 0; e < d1.ne; ++e) f[e] = d1.span[e] - d1.p;
    put(img, L.e1first, f);
    f.assign(d2.ne, 0);
    for (int e = 0; e < d2.ne; ++e) f[e] = d2.span[e] - d2.p;
    put(img, L.e2first, f);
  }
  {
    std::vector<int> pe(2 * d1.pair_elo.size());
    for (size_t i = 0; i < d1.pair_elo.size(); ++i) {
      pe[2 * i] = d1.pair_elo[i];
      pe[2 * i + 1] = d1.pair_ecnt[i];
    }
    put(img, L.pe1, pe);
    pe.assign(2 * d2.pair_elo.size(), 0);
    for (size_t i = 0; i < d2.pair_elo.size(); ++i) {
      pe[2 * i] = d2.pair_elo[i];
      pe[2 * i + 1] = d2.pair_ecnt[i];
    }
    put(img, L.pe2, pe);
  }
  put(img, L.srow, srow);
  put(img, L.krow, krow);
  put(img, L.kcol, kcol);
  put(img, L.kp1, kp1);
  put(img, L.kp2, kp2);
  put(img, L.zfirst, zfirst);
  put(img, L.zply, zply);
  put(img, L.ztab, ztab);
  put(img, L.zw, zw);
  put(img, L.zrow, zrow);
  put(img, L.zcol, zcol);
  put(img, L.zkrow, zkrow);
  put(img, L.zcptr, zcptr);
  put(img, L.zcell, zcell);
  put(img, L.zaptr, zaptr);
  put(img, L.zaset, zaset);
  put(img, L.a1f, a1f);
  put(img, L.a1c, a1c);
  put(img, L.a2f, a2f);
  put(img, L.a2c, a2c);
  put(img, L.zs_first, zs_first);
  put(img, L.zs_cptr, zs_cptr);
  put(img, L.zs_cell, zs_cell);
  put(img, L.rowply, rowply);
  put(img, L.rowfin, rowfin);
  put(img, L.set_mat, set_mat);
  put(img, L.set_aux, set_aux);
  put(img, L.ply_mat, plymat);
  put(img, L.ply_set, ply_set);
  put(img, L.tiles, tiles);
  put(img, L.zchunk, zchunk);
  put(img, L.chunk_ptr, chunk_ptr);
  put(img, L.group_ptr, group_ptr);
  put(img, L.group_sptr, group_sptr);
  put(img, L.group_set, group_set);
  put(img, L.chunk_lset, chunk_lset);
  put(img, L.chunk_sptr, chunk_sptr);
  put(img, L.chunk_set, chunk_set);
  put(img, L.zaslot, zaslot);
  put(img, L.gtab, gtab);
  put(img, L.rtab, rtab);
  *out = P;
  return LAM_OK;
}

}  // namespace lam

namespace lam {
bool tuning_ok(const lam_tuning *t) {
  return !t || (t->tile_k >= 0 && t->tile_k <= 85 && t->target_blocks >= 0 && t->lds_kib >= 0 && t->lds_kib <= 160 &&
                (t->set_slots == 0 || t->set_slots == 1 || t->set_slots == 2 || t->set_slots == 4 ||
                 t->set_slots == 8));
}
}  // namespace lam

extern "C" LAM_API lam_status lam_plan_create(const lam_laminate_desc *d, lam_plan **out) {
  return lam::plan_create(d, nullptr, 1, out);
}

extern "C" LAM_API lam_status lam_plan_create_tuned(const lam_laminate_desc *d, const lam_tuning *tuning,
                                                   lam_plan **out) {
  if (!lam::tuning_ok(tuning)) return LAM_EINVAL;
  return lam::plan_create(d, tuning, 1, out);
}

extern "C" LAM_API lam_status lam_plan_create_shell(const lam_laminate_desc *d, const lam_shell *shell,
                                                   const lam_tuning *tuning, lam_plan **out) {
  if (!shell) return LAM_EINVAL;
  if (!lam::tuning_ok(tuning)) return LAM_EINVAL;
  return lam::plan_create(d, tuning, 1, out, shell);
}

extern "C" LAM_API void lam_plan_destroy(lam_plan *p) { delete p; }

extern "C" LAM_API lam_status lam_plan_info(const lam_plan *p, int64_t *n_rows, int64_t *nnz, int64_t *ws_bytes,
                                            int32_t *n_sets, int32_t *n_ply, int32_t *n_mat) {
  if (!p) return LAM_EINVAL;
  if (n_rows) *n_rows = p->nrows;
  if (nnz) *nnz = p->nnz;
  if (ws_bytes) *ws_bytes = p->L.total;
  if (n_sets) *n_sets = p->n_sets;
  if (n_ply) *n_ply = p->n_ply;
  if (n_mat) *n_mat = p->n_mat;
  return LAM_OK;
}

extern "C" LAM_API const char *lam_status_string(lam_status s) {
  switch (s) {
    case LAM_OK: return "ok";
    case LAM_EINVAL: return "invalid argument";
    case LAM_EKNOT: return "invalid knot vector or degree";
    case LAM_EPLY: return "invalid ply stack";
    case LAM_EMAT: return "invalid material, angle or map gradient";
    case LAM_ESIZE: return "workspace or output size does not match the plan";
    case LAM_EHIP: return "HIP runtime error";
    case LAM_EUNSUP: return "outside the limits of this build";
    case LAM_ESCRATCH: return "the plan's scratch exceeds the static scratch of lam_assemble_static";
    default: return "unknown status";
  }
}

extern "C" LAM_API const char *lam_version(void) { return "lamasm 0.1 (gfx950, FP64)"; }
