// kernels.hip -- gfx950 kernels of the fast 2D x 1D assembly and the device
// entry points of the C ABI.
//
// Path of lam_assemble (all kernels on the caller's stream, FP64):
//   k_rotate   per set: rotated 6x6 D_s (bucket, per ply) or its angular
//              harmonic (harmonic mode), and the 81 coefficients
//              E_s[k][l][r][t] = [B(e_k)^T D_s B(e_l)]_{rt}   (eq. B_1, eq. D)
//   k_prep     per in-plane nonzero: the set-independent moments of grad V
//              and W, each a product of two 1D Gauss sums (eq. P without
//              the material); per thickness nonzero and set slot: the 1D
//              integrals Q_l summed over the set's plies          (eq. Q)
//   k_kron_reg every nonzero of K written once, in CSR order, with
//              P_s = moments x E_s formed in registers:
//              sum_sets sum_ab Qbar ⊗ P                          (eq. Km_2)
// (LDS mode, more than eight sets on a thickness row: k_p2d stores P of
// every set, k_q1d, k_kron_lds.)  Also here: the standard 3D assembly, the
// adjoint and its rank-one form, the matrix-free product and CG, and the
// pattern kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <mutex>

#include "device.h"
#include "internal.h"

namespace {

using lam::Region;
using namespace lamdev;

// One thread per set (rotation) and per ply (its bucket check): the grid covers both.
__global__ void __launch_bounds__(64) k_rotate(Dev d, const double *__restrict__ C, const double *__restrict__ theta) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  check_ply(d, theta, t);
  rotate_one(d, C, theta, t);
}

// Standard assembly: every ply's rotated tensor as bracket coefficients.
__global__ void k_rotate_plies(Dev d, const double *__restrict__ C, const double *__restrict__ theta) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= d.n_ply) return;
  double D[6][6];
  rotate_c(C + 36 * d.ply_mat[l], cos(theta[l]), sin(theta[l]), D);
  bracket_coefficients(D, d.Eply + 81 * l);
}

// Harmonic plans: each ply's tensor is its material's harmonic components
// D_h (from k_rotate) summed with the ply's weights, D_l = sum_h f_h(theta_l) D_h
// (Remark on orientations), and its bracket coefficients go to Eply, where the
// scatter reads them (its sets are the plies).
__global__ void k_harm_ply(Dev d, const double *__restrict__ theta) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= d.n_ply) return;
  const int s0 = d.ply_set[l];  // the material's first harmonic set
  double D[6][6];
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) D[I][J] = 0.0;
  for (int h = 0; h < d.n_harm; ++h) {
    const double w = harmonic_weight(d.n_harm, d.set_aux[s0 + h], theta[l]);
    const double *Dh = d.D + 36 * (s0 + h);
    for (int I = 0; I < 6; ++I)
      for (int J = 0; J < 6; ++J) D[I][J] += w * Dh[6 * I + J];
  }
  bracket_coefficients(D, d.Eply + 81 * l);
}

__global__ void __launch_bounds__(256) k_p2d(Dev d, const double *__restrict__ Ec, double *__restrict__ Pt,
                                             double *__restrict__ Mt, int write_p) {
  p2d_one(d, Ec, Pt, Mt, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, write_p);
}

// four entries per 256-thread block, one per wave
__global__ void __launch_bounds__(256) k_q1d(Dev d, const double *__restrict__ theta) {
  q1d_wave(d, theta, (int64_t)blockIdx.x * 4 + threadIdx.x / 64, threadIdx.x & 63);
}

// Register mode: the 2D moments and the folded 1D coefficients do not depend
// on each other or on the set tensors, so one launch computes both (blocks
// [0, nb_m): moments, a thread per in-plane nonzero; the rest: 1D
// coefficients, a wave per entry).
__global__ void __launch_bounds__(256) k_prep(Dev d, const double *__restrict__ theta, int nb_m) {
  const int b = blockIdx.x;
  if (b < nb_m)
    p2d_one(d, nullptr, nullptr, d.M, (int64_t)b * 256 + threadIdx.x, 0);
  else
    q1d_wave(d, theta, (int64_t)(b - nb_m) * 4 + threadIdx.x / 64, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// Materials that vary over the plane (Assumption 3): C_m(xi) = sum_i R^i(xi) C_{m,i}.
// The rotation by the set's angle and the bracket coefficients are linear in
// C, so each set's coefficients at a Gauss point are the basis-weighted sum of
// its coefficients at the in-plane functions; P of each set is the 2D Gauss
// sum of eq. P with that point's coefficients inside.  Three launches:

// per (set, in-plane function): Ectl[s][i] = brackets of T(theta_s) C_{m(s),i} T^T
__global__ void __launch_bounds__(256) k_rotate_field(Dev d, const double *__restrict__ C,
                                                      const double *__restrict__ theta) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)d.n_sets * d.ns) return;
  const int s = (int)(idx / d.ns), c = (int)(idx % d.ns);
  const double *Cm = C + 36 * ((int64_t)d.set_mat[s] * d.ns + c);
  if (idx < d.n_ply) check_ply(d, theta, (int)idx);
  const double th = theta[d.set_aux[s]];
  double D[6][6];
  rotate_c(Cm, cos(th), sin(th), D);
  bracket_coefficients(D, d.Ectl + 81 * idx);
}

// per (set, in-plane element, Gauss point, coefficient j):
// Epts[s][e][g][j] = sum_b R_b(e, g) Ectl[s][function b of e][j]
__global__ void __launch_bounds__(256) k_field_points(Dev d) {
  const int64_t npts = (int64_t)d.ne1 * d.ne2 * d.ngp;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 81 * npts * d.n_sets) return;
  const int j = (int)(idx % 81);
  const int64_t pt = idx / 81, s = pt / npts, rem = pt % npts;
  const int64_t e = rem / d.ngp;
  const int e1 = (int)(e % d.ne1), e2 = (int)(e / d.ne1), P1 = d.p1 + 1;
  const int f1 = d.e1first[e1], f2 = d.e2first[e2];
  const double *R = d.rtab + rem * d.nb * 3;
  const double *Es = d.Ectl + 81 * s * d.ns;
  double acc = 0.0;
  for (int b = 0; b < d.nb; ++b) {
    const int is = (f2 + b / P1) * d.n1 + f1 + b % P1;
    acc += R[3 * b] * Es[81 * (int64_t)is + j];
  }
  d.Epts[81 * pt + j] = acc;
}

// P of every set with the material field inside (Assumption 3), element by
// element: one block per (in-plane element e, set s) stages the element's
// point data in LDS (the map gradient and weight, the (rational) basis values
// and derivatives of its nb local functions, and the set's bracket
// coefficients E_s at every point), and each thread takes local pairs (a, b)
// and adds
//   P_s[k(a, b)][ab][rt] += sum_g w_g |DF| sum_kl (G_a)_k (G_b)_l E_s(g)[kl][rt]
// into the pair's in-plane nonzero k (stored component-major for the
// LDS-mode scatter), the E reads broadcast across the block.
// Elements of one colour (e1 mod p1 + 1, e2 mod p2 + 1) share no in-plane
// function, so a launch per colour adds without atomics (P zeroed first).
__global__ void __launch_bounds__(256) k_p2d_field(Dev d, int c1, int c2, int n1c, int n2c) {
  extern __shared__ double fs[];
  const int P1 = d.p1 + 1, P2 = d.p2 + 1, nb = P1 * P2, ngp = d.ngp;
  const int64_t blk = blockIdx.x;
  const int s = (int)(blk / ((int64_t)n1c * n2c));
  const int eb = (int)(blk - (int64_t)s * n1c * n2c);
  const int e1 = c1 + P1 * (eb % n1c), e2 = c2 + P2 * (eb / n1c);
  const int64_t e = e1 + (int64_t)d.ne1 * e2;
  const int64_t npts = (int64_t)d.ne1 * d.ne2 * ngp;
  double *sG = fs, *sR = sG + 10 * ngp, *sE = sR + 3 * nb * ngp;  // [g][10], [g][nb][3], [g][81]
  for (int x = threadIdx.x; x < 10 * ngp; x += blockDim.x) sG[x] = d.gtab[e * ngp * 10 + x];
  for (int x = threadIdx.x; x < 3 * nb * ngp; x += blockDim.x) sR[x] = d.rtab[e * ngp * nb * 3 + x];
  for (int x = threadIdx.x; x < 81 * ngp; x += blockDim.x) sE[x] = d.Epts[81 * (s * npts + e * ngp) + x];
  __syncthreads();
  const int f1 = d.e1first[e1], f2 = d.e2first[e2];
  for (int u = threadIdx.x; u < nb * nb; u += blockDim.x) {
    const int la = u / nb, lb = u - la * nb;
    double P[4][9];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab)
#pragma unroll
      for (int rt = 0; rt < 9; ++rt) P[ab][rt] = 0.0;
    for (int g = 0; g < ngp; ++g) {
      const double *G = sG + 10 * g, *ri = sR + 3 * (g * nb + la), *rj = sR + 3 * (g * nb + lb);
      const double *E = sE + 81 * g;
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
          const double *Ekl = E + 9 * (kk * 3 + ll);
          double ek[9];
#pragma unroll
          for (int rt = 0; rt < 9; ++rt) ek[rt] = Ekl[rt];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              const double m = w * vi[a][kk] * vj[b][ll];
#pragma unroll
              for (int rt = 0; rt < 9; ++rt) P[2 * a + b][rt] += m * ek[rt];
            }
        }
    }
    // the pair's in-plane nonzero: row is = i1 + n1 i2, column js = j1 + n1 j2
    const int i1 = f1 + la % P1, i2 = f2 + la / P1, j1 = f1 + lb % P1, j2 = f2 + lb / P1;
    const int64_t k = d.srow[i1 + d.n1 * i2] + (int64_t)(j2 - d.a2f[i2]) * d.a1c[i1] + (j1 - d.a1f[i1]);
    // read-modify-write of the pair's 36 entries (distinct, one per component
    // plane), nine at a time with every read of a batch issued before its
    // first write: a read after a write also waits for that write (one counter
    // for both), so entry by entry would serialize 36 round trips
    double *Po = d.P + (int64_t)s * 36 * d.nnz2 + k;
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) {
      double *Pab = Po + (int64_t)(ab * 9) * d.nnz2;
      double old[9];
#pragma unroll
      for (int rt = 0; rt < 9; ++rt) old[rt] = Pab[(int64_t)rt * d.nnz2];
#pragma unroll
      for (int rt = 0; rt < 9; ++rt) Pab[(int64_t)rt * d.nnz2] = old[rt] + P[ab][rt];
    }
  }
}

// ---------------------------------------------------------------------------
// CSR addressing.  Row (it, is, r) starts at
//   9*nnz2*zrow[it] + 3*Lz(it)*(3*srow[is] + r*Ls(is))
// and its entry for thickness column a (0..Lz-1), in-plane column b
// (0..Ls-1) and component t sits at + a*3*Ls + 3*b + t: columns ascend in
// (jt, js, t) because both 1D overlap lists are contiguous and ascending.

// Kronecker scatter.  Block = (tile of whole in-plane rows, chunk of
// thickness rows); the blocks of each XCD (block ids congruent mod 8) take a
// contiguous range of tiles.  For every thickness row it the tile's output is
// one contiguous range of the CSR values: rows is of the tile, then r, then
// thickness column a, then in-plane column b, then t.  Thread = one
// (in-plane nonzero k, component t) slot, consecutive slots on consecutive
// lanes; it computes
//   out = sum_j sum_ab Qc[zk][j][ab] * P[set_j][k][ab][r][t]
// for all (r, a) with P of the chunk's sets and the chunk's coefficients Qc
// staged in LDS (so that no global load is waited on while stores are in
// flight), then stores r-major, a-minor: consecutive store instructions of a
// wave write adjacent runs, so each CSR row is written front to back as one
// sequential stream.
// Block -> (tile, group of chunks): consecutive blocks go to the eight XCDs in
// turn, so each XCD takes a contiguous range of tiles and walks its groups in
// thickness order.
__device__ inline int kron_block(const Dev &d, int &tile, int &g) {
  const int nblk = d.n_tiles * d.n_groups;
  const int per = (nblk + 7) / 8;
  const int L = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  tile = L / d.n_groups;
  g = L - tile * d.n_groups;
  return L < nblk;
}

template <bool USE_LDS>
__global__ void __launch_bounds__(KRON_THREADS) k_kron_lds(Dev d, double *__restrict__ vals) {
  extern __shared__ double lds[];
  int tile, g;
  if (!kron_block(d, tile, g)) return;
  const int ch = d.group_ptr[g];  // the planner gives LDS mode one chunk per group
  const int k0 = d.tiles[tile], tk = d.tiles[tile + 1] - k0;
  const int it0 = d.chunk_ptr[ch], it1 = d.chunk_ptr[ch + 1];
  const int zk0 = d.zrow[it0], nzk = d.zrow[it1] - zk0;
  const int c0 = d.chunk_sptr[ch], nsc = d.chunk_sptr[ch + 1] - c0;
  const int per_set = 36 * tk;
  double *lq = lds;                     // [nzk][maxact][4]
  double *lp = lds + d.kron_lds_q / 8;  // [nsc][tk][36]
  for (int e = threadIdx.x; e < 4 * d.maxact * nzk; e += KRON_THREADS) lq[e] = d.Qc[4 * (int64_t)d.maxact * zk0 + e];
  if (USE_LDS) {
    for (int e = threadIdx.x; e < nsc * per_set; e += KRON_THREADS) {
      // read k-fastest from the component-major table, store [slot][k][36]
      const int sc = e / per_set, rem = e - sc * per_set, comp = rem / tk, kk = rem - comp * tk;
      lp[(sc * tk + kk) * 36 + comp] = d.P[((int64_t)d.chunk_set[c0 + sc] * 36 + comp) * d.nnz2 + k0 + kk];
    }
  }
  __syncthreads();
  const int sig = threadIdx.x;
  if (sig >= 3 * tk) return;
  const int kk = sig / 3, t = sig - 3 * kk, k = k0 + kk;
  const int is = d.krow[k], sr = d.srow[is];
  const int Ls = d.srow[is + 1] - sr, off = 3 * (k - sr) + t;
  const int64_t astride = 3 * (int64_t)Ls;
  for (int it = it0; it < it1; ++it) {
    const int zb = d.zrow[it], Lz = d.zrow[it + 1] - zb;
    const int a0 = d.zaptr[it], na = d.zaptr[it + 1] - a0;
    double *out = vals + 9 * d.nnz2 * (int64_t)zb + 9 * (int64_t)Lz * sr + off;
    const int64_t rstride = 3 * (int64_t)Lz * Ls;
    for (int ab0 = 0; ab0 < Lz; ab0 += KRON_AB) {
      double acc[KRON_AB][3];
#pragma unroll
      for (int x = 0; x < KRON_AB; ++x) acc[x][0] = acc[x][1] = acc[x][2] = 0.0;
      for (int j = 0; j < na; ++j) {
        double pr[4][3];
        if (USE_LDS) {
          const double *Pp = lp + (d.zaslot[a0 + j] * tk + kk) * 36 + t;
#pragma unroll
          for (int ab = 0; ab < 4; ++ab)
#pragma unroll
            for (int r = 0; r < 3; ++r) pr[ab][r] = Pp[ab * 9 + 3 * r];
        } else {
          const double *Pp = d.P + (int64_t)d.zaset[a0 + j] * 36 * d.nnz2 + k;
#pragma unroll
          for (int ab = 0; ab < 4; ++ab)
#pragma unroll
            for (int r = 0; r < 3; ++r) pr[ab][r] = Pp[(int64_t)(ab * 9 + 3 * r + t) * d.nnz2];
        }
#pragma unroll
        for (int x = 0; x < KRON_AB; ++x) {
          if (ab0 + x < Lz) {
            const double *qq = lq + 4 * ((zb + ab0 + x - zk0) * d.maxact + j);
            const double q0 = qq[0], q1 = qq[1], q2 = qq[2], q3 = qq[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) acc[x][r] += q0 * pr[0][r] + q1 * pr[1][r] + q2 * pr[2][r] + q3 * pr[3][r];
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
}

// Register mode of the scatter.
//  - one or two set slots (every bucket and per-ply plan): one block per
//    (tile, group of chunks).  The block stages the bracket coefficients of
//    the group's sets in LDS behind one barrier; then per chunk each thread
//    contracts P of the chunk's slots for its (k, t) into registers and writes
//    the chunk's rows, the rows' coefficients read through scalar loads.
//    After the barrier the block issues no vector loads, so no wait on a load
//    also waits for the stores in flight, and the stores stream.
//  - four or eight slots: one block per (tile, chunk) (the planner gives each
//    group one chunk), P of the slots in registers, coefficients in LDS.
// P at (k, t) is contracted from the set-independent moments M_ab[kl] (one
// table for all sets) and a slot's bracket coefficients E_s[kl][rt] (eq. P):
// P is never stored.  FIELD (one or two slots, materials varying over the
// plane): P of every set is stored and read per set change instead.
template <int NSC, bool FIELD>
__global__ void __launch_bounds__(KRON_THREADS) k_kron_reg(Dev d, const double *__restrict__ qd,
                                                           double *__restrict__ vals) {
  // LDS: slot-dense coefficients [zk - zk0][NSC][4] (kron_lds_q bytes; left
  // unused by the one- and two-slot path, which reads them through scalar
  // loads), then bracket coefficients [81] per set of the group and one zero
  // block (or per slot)
  extern __shared__ double lq[];
  int tile, g;
  if (!kron_block(d, tile, g)) return;
  if constexpr (NSC <= 2) {
    lamdev::kron_group<NSC, FIELD>(d, qd, vals, tile, g, lq, (int)threadIdx.x, (int)blockDim.x);
  } else {
    const int k0 = d.tiles[tile], tk = d.tiles[tile + 1] - k0;
    const int sig = threadIdx.x;
    const bool act = sig < 3 * tk;
    const int kk = act ? sig / 3 : 0, t = act ? sig - 3 * kk : 0, k = k0 + kk;
    double mv[4][9];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab)
#pragma unroll
      for (int kl = 0; kl < 9; ++kl) mv[ab][kl] = d.M[m_index(k, ab * 9 + kl)];
    const int is = d.krow[k], sr = d.srow[is];
    const int Ls = d.srow[is + 1] - sr, off = 3 * (k - sr) + t;
    const int64_t astride = 3 * (int64_t)Ls;
    double *le = lq + d.kron_lds_q / 8;
    const int ch = d.group_ptr[g];
    const int it0 = d.chunk_ptr[ch], it1 = d.chunk_ptr[ch + 1];
    const int zk0 = d.zrow[it0], nq = 4 * NSC * (d.zrow[it1] - zk0);
    const int c0 = d.chunk_sptr[ch], nsc = d.chunk_sptr[ch + 1] - c0;
    for (int e = sig; e < NSC * 81; e += blockDim.x) {
      const int u = e / 81;
      le[e] = u < nsc ? d.Escat[81 * (int64_t)d.chunk_set[c0 + u] + (e - 81 * u)] : 0.0;
    }
    for (int e = sig; e < nq; e += blockDim.x) lq[e] = qd[4 * (int64_t)NSC * zk0 + e];
    __syncthreads();
    if (!act) return;
    double pr[NSC][4][3];
#pragma unroll
    for (int u = 0; u < NSC; ++u)
#pragma unroll
      for (int ab = 0; ab < 4; ++ab)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          double a = 0.0;
#pragma unroll
          for (int kl = 0; kl < 9; ++kl) a += mv[ab][kl] * le[81 * u + kl * 9 + 3 * r + t];
          pr[u][ab][r] = a;
        }
    for (int it = it0; it < it1; ++it) {
      const int zb = d.zrow[it], Lz = d.zrow[it + 1] - zb;
      double *out = vals + 9 * d.nnz2 * (int64_t)zb + 9 * (int64_t)Lz * sr + off;
      const int64_t rstride = 3 * (int64_t)Lz * Ls;
      for (int ab0 = 0; ab0 < Lz; ab0 += KRON_AB) {
        double acc[KRON_AB][3];
#pragma unroll
        for (int x = 0; x < KRON_AB; ++x) {
          acc[x][0] = acc[x][1] = acc[x][2] = 0.0;
          if (ab0 + x < Lz) {
            const double *qq = lq + 4 * NSC * (zb + ab0 + x - zk0);
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
  }
}

// ---------------------------------------------------------------------------
// Matrix-free product y = K u (eq. Km_2 applied to a vector; K is never
// formed).  Same blocks as the register-mode scatter (a tile of whole in-plane
// rows x a group of thickness chunks, one or two set slots) and the same P in
// registers per chunk; for every thickness row it of the group each thread
// (k = (is, js), t) first contracts the row's thickness coefficients with u,
//   V_u[ab] = sum_x Qd[zk_x][u][ab] u[3 (jt_x n_s + js) + t],
// then forms its share c_r = sum_u sum_ab P_u[ab][r] V_u[ab] of
// y[3 (it n_s + is) + r].  The shares of APPLY_ROWS thickness rows go to LDS
// behind one barrier and are summed per (row, in-plane row, r) by one thread
// each, in three chains (one per component t) so the LDS reads overlap; every
// entry of y belongs to exactly one block, so no atomics.
// fixed (nullable, one byte per row): Dirichlet elimination, y = P K P u +
// (I - P) u with P the projection on the free rows (fixed entries of u read
// as 0, fixed rows of y copy u).  FIELD (in-plane material fields): each
// slot's P is read from the stored P of its set instead of formed from the
// moments, as in the scatter.
constexpr int APPLY_ROWS = 8;

template <int NSC, bool FIELD>
__global__ void __launch_bounds__(KRON_THREADS) k_apply(Dev d, const double *__restrict__ qd,
                                                        const double *__restrict__ u,
                                                        const uint8_t *__restrict__ fixed, double *__restrict__ y) {
  static_assert(NSC <= 2, "the matrix-free product keeps at most two set slots");
  // LDS: group coefficients (kron_lds_q bytes), set brackets (kron_lds_p
  // bytes), then the shares c[APPLY_ROWS][3][3 tile_k] (one slot per active thread)
  extern __shared__ double lq[];
  int tile, g;
  if (!kron_block(d, tile, g)) return;
  const int k0 = d.tiles[tile], tk = d.tiles[tile + 1] - k0;
  const int sig = threadIdx.x, nth = blockDim.x;
  const bool act = sig < 3 * tk;
  const int kk = act ? sig / 3 : 0, t = act ? sig - 3 * kk : 0, k = k0 + kk;
  double mv[4][9];  // the moments (material fields read their stored P instead)
  if constexpr (!FIELD) {
#pragma unroll
    for (int ab = 0; ab < 4; ++ab)
#pragma unroll
      for (int kl = 0; kl < 9; ++kl) mv[ab][kl] = d.M[m_index(k, ab * 9 + kl)];
  }
  const int js = d.kcol[k];
  const int is0 = d.krow[k0], nrow = d.krow[k0 + tk - 1] - is0 + 1;  // the tile's in-plane rows
  const int ch0 = d.group_ptr[g], ch1 = d.group_ptr[g + 1];
  const int itg0 = d.chunk_ptr[ch0], itg1 = d.chunk_ptr[ch1];
  const int zk0 = d.zrow[itg0], nq = 4 * NSC * (d.zrow[itg1] - zk0);
  const int s0 = d.group_sptr[g], ns = d.group_sptr[g + 1] - s0;
  double *le = lq + d.kron_lds_q / 8;
  const int ns3 = 3 * d.tile_k;          // share slots per row: the plan's widest tile
  double *lc = le + d.kron_lds_p / 8;  // [APPLY_ROWS][3][ns3]
  for (int e = sig; e < 81 * (ns + 1); e += nth) {
    const int w = e / 81;
    le[e] = w < ns ? d.Escat[81 * (int64_t)d.group_set[s0 + w] + (e - 81 * w)] : 0.0;
  }
  for (int e = sig; e < nq; e += nth) lq[e] = qd[4 * (int64_t)NSC * zk0 + e];
  __syncthreads();
  double pr[NSC][4][3];
  // material fields: group-local set of each slot's P, so that a slot whose
  // set the previous chunk also had (the planner keeps it in place) is not
  // read again.  Not for constant materials: there P is a few FMAs from
  // registers and LDS, and the tracking registers cost the two-slot kernel a
  // wave per SIMD (167 -> 182 VGPRs; the 64x64 32-ply product 0.25 -> 0.32 ms).
  int slot_set[NSC];
#pragma unroll
  for (int w = 0; w < NSC; ++w) slot_set[w] = -1;
  int ch = ch0 - 1, ch_end = itg0;  // chunk of the current row; its last row + 1
  for (int b0 = itg0; b0 < itg1; b0 += APPLY_ROWS) {  // block-uniform trip counts and barriers
    const int nb = itg1 - b0 < APPLY_ROWS ? itg1 - b0 : APPLY_ROWS;
    for (int j = 0; j < nb; ++j) {
      const int it = b0 + j;
      while (it >= ch_end) {  // entering the next chunk: P of its slots
        ++ch;
        ch_end = d.chunk_ptr[ch + 1];
        const int c0 = d.chunk_sptr[ch], nsc = d.chunk_sptr[ch + 1] - c0;
#pragma unroll
        for (int w = 0; w < NSC; ++w) {
          const int ls = w < nsc ? d.chunk_lset[c0 + w] : ns;  // unused slots: the zero block
          if constexpr (FIELD) {
            if (ls == slot_set[w]) continue;  // the slot keeps its set (and P) from the previous chunk
            slot_set[w] = ls;
            const int gs = ls < ns ? d.group_set[s0 + ls] : -1;
#pragma unroll
            for (int ab = 0; ab < 4; ++ab)
#pragma unroll
              for (int r = 0; r < 3; ++r)
                pr[w][ab][r] = act && gs >= 0 ? d.P[((int64_t)gs * 36 + ab * 9 + 3 * r + t) * d.nnz2 + k] : 0.0;
            continue;
          }
          const double *ew = le + 81 * ls;
#pragma unroll
          for (int ab = 0; ab < 4; ++ab)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
              double a = 0.0;
#pragma unroll
              for (int kl = 0; kl < 9; ++kl) a += mv[ab][kl] * ew[kl * 9 + 3 * r + t];
              pr[w][ab][r] = act ? a : 0.0;
            }
        }
      }
      const int zb = d.zrow[it], Lz = d.zrow[it + 1] - zb;
      double v[NSC][4];
#pragma unroll
      for (int w = 0; w < NSC; ++w) v[w][0] = v[w][1] = v[w][2] = v[w][3] = 0.0;
      for (int x = 0; x < Lz; ++x) {
        const int64_t col = 3 * ((int64_t)d.zcol[zb + x] * d.ns + js) + t;
        const double ux = fixed && fixed[col] ? 0.0 : u[col];
        const double *q = lq + 4 * NSC * (zb + x - zk0);
#pragma unroll
        for (int w = 0; w < NSC; ++w)
#pragma unroll
          for (int ab = 0; ab < 4; ++ab) v[w][ab] += q[4 * w + ab] * ux;
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        double c = 0.0;
#pragma unroll
        for (int w = 0; w < NSC; ++w)
#pragma unroll
          for (int ab = 0; ab < 4; ++ab) c += pr[w][ab][r] * v[w][ab];
        if (sig < ns3) lc[(3 * j + r) * ns3 + sig] = c;
      }
    }
    __syncthreads();
    for (int o = sig; o < 3 * nrow * nb; o += nth) {
      const int j = o / (3 * nrow), rem = o - 3 * nrow * j, i = rem / 3, r = rem - 3 * i, is = is0 + i;
      const int m0 = d.srow[is] - k0, m1 = d.srow[is + 1] - k0;
      const double *src = lc + (3 * j + r) * ns3;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
      for (int m = m0; m < m1; ++m) {
        a0 += src[3 * m];
        a1 += src[3 * m + 1];
        a2 += src[3 * m + 2];
      }
      const double acc = (a0 + a1) + a2;
      const int64_t row = 3 * ((int64_t)(b0 + j) * d.ns + is) + r;
      y[row] = fixed && fixed[row] ? u[row] : acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Standard 3D assembly (the comparator of the method, Sec. 2.4).  A 3D element
// is (in-plane element e1, e2) x (thickness knot span) with the ply cells
// inside the span.
//
// With the ply tensor constant in a cell, the element matrix of the cell is
//   K_ab[r][t] = sum_kl M_kl(a, b) E[kl][rt],  M_kl(a, b) = sum_g w_g G_a(g)_k G_b(g)_l,
// G_a(g) the physical gradient of local function a at Gauss point g and E the
// ply's bracket coefficients.  M is a dense product over the points, done on
// the FP64 matrix cores: the nloc local functions are cut into 16-wide tiles
// and a wavefront takes one tile pair (I <= J) of an element at a time,
// running the nine chains M_kl (k, l = 0..2) of v_mfma_f64_16x16x4f64, four
// points per step: lane i + 16 kk holds the operands w G_a(g)_k for
// a = 16 I + i and G_b(g)_l for b = 16 J + i at point g = 4 s + kk (read from
// a gradient table the block builds in LDS, or evaluated in the lane from
// the 1D or shell basis tables).  After each ply cell the
// nine M tiles are contracted with that ply's E into the element matrix,
// which is added to the CSR once: the tile (I, J) as K_ab and, for I < J, its
// transpose as K_ba (K is symmetric: E[kl][rt] = E[lk][tr]).  Padded
// functions and points carry zero operands.
//
// The adds are plain read-modify-writes, conflict-free by colouring (one
// launch per colour: e1 mod p1 + 1, e2 mod p2 + 1, span mod q + 1; elements
// of one colour share no basis function), so the result does not depend on
// the schedule.

// v_mfma_f64_16x16x4f64 leaves D[lane / 16 + 4 v][lane % 16] in item v of the lane
typedef double std_dbl4 __attribute__((ext_vector_type(4)));
constexpr int STD_WAVES = 4;      // wavefronts (tile pairs) per block, operands from the tables
constexpr int STD_LDS_WAVES = 8;  // most tile pairs (one wavefront each) of the LDS-table kernel

__global__ void k_fill_zero(double *__restrict__ v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = 0.0;
}

// physical gradient of local function (a1, a2, at) at point (g1, g2, gz) of cell c
// of in-plane element (e1, e2), and the point's weight (in-plane, |DF|, thickness)
__device__ inline void std_gradient(const Dev &d, int e1, int e2, int c, int g1, int g2, int gz, int a1, int a2, int at,
                                    double G[3], double &w) {
  const int P1 = d.p1 + 1, Q1 = d.q + 1;
  const double *t3 = d.ztab + (((int64_t)c * d.ngz + gz) * Q1 + at) * 2;
  double gh[3];
  const double *Jt;
  if (d.shell) {
    const int64_t ep = ((int64_t)e1 + (int64_t)d.ne1 * e2) * d.ngp + g1 + d.ng1 * g2;
    const double *rt = d.rtab + (ep * d.nb + a1 + P1 * a2) * 3;
    gh[0] = rt[1] * t3[0];
    gh[1] = rt[2] * t3[0];
    gh[2] = rt[0] * t3[1];
    Jt = d.gtab + ep * 10;
    w = Jt[9];
  } else {
    const int P2 = d.p2 + 1;
    const double *t1 = d.tab1 + (((int64_t)e1 * d.ng1 + g1) * P1 + a1) * 2;
    const double *t2 = d.tab2 + (((int64_t)e2 * d.ng2 + g2) * P2 + a2) * 2;
    gh[0] = t1[1] * t2[0] * t3[0];
    gh[1] = t1[0] * t2[1] * t3[0];
    gh[2] = t1[0] * t2[0] * t3[1];
    Jt = d.jit;
    w = d.w1[(int64_t)e1 * d.ng1 + g1] * d.w2[(int64_t)e2 * d.ng2 + g2] * d.detj;
  }
  w *= d.zw[(int64_t)c * d.ngz + gz];
#pragma unroll
  for (int k = 0; k < 3; ++k) G[k] = Jt[k * 3 + 0] * gh[0] + Jt[k * 3 + 1] * gh[1] + Jt[k * 3 + 2] * gh[2];
}

// the CSR entry of (row function i, component r) x (column function j, component t):
// returns the address of component (r, t) = (0, 0); r steps by rstride, t by 1
__device__ inline double *std_entry(const Dev &d, double *vals, int i1, int i2, int it, int j1, int j2, int jt,
                                    int64_t &rstride) {
  const int is = i1 + d.n1 * i2;
  const int zb = d.zrow[it], Lz = d.zrow[it + 1] - zb;
  const int sr = d.srow[is], Ls = d.srow[is + 1] - sr;
  const int az = jt - d.zcol[zb];
  const int bs = (j2 - d.a2f[i2]) * d.a1c[i1] + (j1 - d.a1f[i1]);
  rstride = 3 * (int64_t)Lz * Ls;
  return vals + 9 * d.nnz2 * (int64_t)zb + 3 * (int64_t)Lz * 3 * sr + (int64_t)az * 3 * Ls + 3 * bs;
}

// ke[v] += sum_kl m[kl][v] E[kl][.]: the nine M tiles of one ply cell contracted
// with its bracket coefficients
__device__ inline void std_contract(const std_dbl4 m[9], const double *E, double ke[4][9]) {
#pragma unroll
  for (int kl = 0; kl < 9; ++kl)
#pragma unroll
    for (int rt = 0; rt < 9; ++rt) {
      const double e = E[kl * 9 + rt];
#pragma unroll
      for (int v = 0; v < 4; ++v) ke[v][rt] += m[kl][v] * e;
    }
}

// Adds the lane's blocks of tile pair (I, J) of element (e1, e2, zsp) into the
// CSR: K_ab for b = 16 J + li and a = 16 I + kk + 4 v, and for I < J the
// transposes K_ba.  Every (v, r, t) entry of the lane, direct or transposed,
// is a distinct CSR position (the pairs differ, and for I < J the transposed
// rows lie in tile J, the direct ones in tile I), so all reads of a block are
// issued before any write: one memory round trip per block instead of one
// per row.
__device__ inline void std_add(const Dev &d, double *__restrict__ vals, int e1, int e2, int zsp, int I, int J,
                               const double ke[4][9]) {
  const int lane = threadIdx.x & 63, li = lane & 15, kk = lane >> 4;
  const int P1 = d.p1 + 1, P2 = d.p2 + 1, Q1 = d.q + 1, nloc = P1 * P2 * Q1;
  const int b = 16 * J + li;
  if (b >= nloc) return;
  const int f1 = d.e1first[e1], f2 = d.e2first[e2], fz = d.zs_first[zsp];
  const int j1 = f1 + b % P1, j2 = f2 + (b / P1) % P2, jt = fz + b / (P1 * P2);
  const int nv = min(4, (nloc - 16 * I - kk + 3) / 4);  // rows a = 16 I + kk + 4 v < nloc of the lane
  double *rowp[4];
  int64_t rstr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = min(16 * I + kk + 4 * v, nloc - 1);  // past the last function: a valid address, not written
    const int i1 = f1 + a % P1, i2 = f2 + (a / P1) % P2, it = fz + a / (P1 * P2);
    rowp[v] = std_entry(d, vals, i1, i2, it, j1, j2, jt, rstr[v]);
  }
  {
    double old[4][9];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (v < nv)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int t = 0; t < 3; ++t) old[v][r * 3 + t] = rowp[v][r * rstr[v] + t];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (v < nv)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int t = 0; t < 3; ++t) rowp[v][r * rstr[v] + t] = old[v][r * 3 + t] + ke[v][r * 3 + t];
  }
  if (I == J) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = min(16 * I + kk + 4 * v, nloc - 1);
    const int i1 = f1 + a % P1, i2 = f2 + (a / P1) % P2, it = fz + a / (P1 * P2);
    rowp[v] = std_entry(d, vals, j1, j2, jt, i1, i2, it, rstr[v]);
  }
  double old[4][9];
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (v < nv)
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 3; ++r) old[v][t * 3 + r] = rowp[v][t * rstr[v] + r];
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (v < nv)
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 3; ++r) rowp[v][t * rstr[v] + r] = old[v][t * 3 + r] + ke[v][r * 3 + t];
}

// std_add in two halves for callers that can issue the reads early: the
// direct block's CSR values (K_ab's entries) are read before the element
// matrix exists (their addresses do not depend on it), so the read latency
// overlaps the products; std_add_late then adds and writes them and does the
// transposed block as std_add does.
__device__ inline void std_add_early(const Dev &d, const double *__restrict__ vals, int e1, int e2, int zsp, int I,
                                     int J, double old[4][9]) {
  const int lane = threadIdx.x & 63, li = lane & 15, kk = lane >> 4;
  const int P1 = d.p1 + 1, P2 = d.p2 + 1, Q1 = d.q + 1, nloc = P1 * P2 * Q1;
  const int b = min(16 * J + li, nloc - 1);  // padded lanes read a valid entry and never write it
  const int f1 = d.e1first[e1], f2 = d.e2first[e2], fz = d.zs_first[zsp];
  const int j1 = f1 + b % P1, j2 = f2 + (b / P1) % P2, jt = fz + b / (P1 * P2);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = min(16 * I + kk + 4 * v, nloc - 1);
    const int i1 = f1 + a % P1, i2 = f2 + (a / P1) % P2, it = fz + a / (P1 * P2);
    int64_t rs;
    const double *row = std_entry(d, const_cast<double *>(vals), i1, i2, it, j1, j2, jt, rs);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int t = 0; t < 3; ++t) old[v][r * 3 + t] = row[r * rs + t];
  }
}

__device__ inline void std_add_late(const Dev &d, double *__restrict__ vals, int e1, int e2, int zsp, int I, int J,
                                    const double ke[4][9], const double old[4][9]) {
  const int lane = threadIdx.x & 63, li = lane & 15, kk = lane >> 4;
  const int P1 = d.p1 + 1, P2 = d.p2 + 1, Q1 = d.q + 1, nloc = P1 * P2 * Q1;
  const int b = 16 * J + li;
  if (b >= nloc) return;
  const int f1 = d.e1first[e1], f2 = d.e2first[e2], fz = d.zs_first[zsp];
  const int j1 = f1 + b % P1, j2 = f2 + (b / P1) % P2, jt = fz + b / (P1 * P2);
  const int nv = min(4, (nloc - 16 * I - kk + 3) / 4);
  double *rowp[4];
  int64_t rstr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = min(16 * I + kk + 4 * v, nloc - 1);
    const int i1 = f1 + a % P1, i2 = f2 + (a / P1) % P2, it = fz + a / (P1 * P2);
    rowp[v] = std_entry(d, vals, i1, i2, it, j1, j2, jt, rstr[v]);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (v < nv)
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int t = 0; t < 3; ++t) rowp[v][r * rstr[v] + t] = old[v][r * 3 + t] + ke[v][r * 3 + t];
  if (I == J) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = min(16 * I + kk + 4 * v, nloc - 1);
    const int i1 = f1 + a % P1, i2 = f2 + (a / P1) % P2, it = fz + a / (P1 * P2);
    rowp[v] = std_entry(d, vals, j1, j2, jt, i1, i2, it, rstr[v]);
  }
  double ot[4][9];
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (v < nv)
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 3; ++r) ot[v][t * 3 + r] = rowp[v][t * rstr[v] + r];
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (v < nv)
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 3; ++r) rowp[v][t * rstr[v] + r] = ot[v][t * 3 + r] + ke[v][r * 3 + t];
}

// tile pair u (0 <= u < tiles (tiles + 1) / 2) -> (I, J), I <= J
__device__ inline void std_pair(int tiles, int u, int &I, int &J) {
  I = 0;
  while (u >= tiles - I) u -= tiles - I++;
  J = I + u;
}

// Element (e1, e2, zsp) for launch index el of colour (c1, c2, c3): elements
// c1 + (p1 + 1) k1, c2 + (p2 + 1) k2, spans c3 + (q + 1) k3, n1c x n2c of them
// per span row.
__device__ inline void std_element(const Dev &d, int64_t el, int c1, int c2, int c3, int n1c, int n2c, int &e1, int &e2,
                                   int &zsp) {
  e1 = c1 + (d.p1 + 1) * (int)(el % n1c);
  e2 = c2 + (d.p2 + 1) * (int)((el / n1c) % n2c);
  zsp = c3 + (d.q + 1) * (int)(el / ((int64_t)n1c * n2c));
}

// blocks round-robin over the 8 XCDs: XCD x takes the x-th contiguous range
// (the grid is a multiple of 8 blocks, so this is a permutation)
__device__ inline int64_t std_block() {
  const int64_t per = gridDim.x / 8;
  return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// Elements of one ply cell, at most eight tile pairs: the block (one
// wavefront per tile pair) builds the element's gradient table in LDS,
// G[g][k][a] (row stride gs doubles per point, padded so the four point rows
// a step reads fall in different banks) and W[g], then every wavefront runs
// its tile pair with the operands read from LDS.
__global__ void __launch_bounds__(64 * STD_LDS_WAVES, 2) k_std3d_lds(Dev d, double *__restrict__ vals, int c1, int c2,
                                                                   int c3, int n1c, int n2c, int64_t n_elem, int tiles,
                                                                   int nlocp, int gs) {
  extern __shared__ double sm[];
  const int64_t el = std_block();
  if (el >= n_elem) return;  // the whole block
  int e1, e2, zsp;
  std_element(d, el, c1, c2, c3, n1c, n2c, e1, e2, zsp);
  const int P1 = d.p1 + 1, P2 = d.p2 + 1;
  const int nloc = P1 * P2 * (d.q + 1), ng = d.ng1 * d.ng2 * d.ngz, nsteps = (ng + 3) / 4, ngp = 4 * nsteps;
  double *G = sm, *W = sm + (int64_t)ngp * gs;
  const int c = d.zs_cell[d.zs_cptr[zsp]];
  for (int idx = threadIdx.x; idx < ngp * nlocp; idx += blockDim.x) {
    const int g = idx / nlocp, a = idx - g * nlocp;
    double Gv[3] = {0.0, 0.0, 0.0}, w = 0.0;
    if (g < ng && a < nloc) {
      const int g1 = g % d.ng1, g2 = (g / d.ng1) % d.ng2, gz = g / (d.ng1 * d.ng2);
      std_gradient(d, e1, e2, c, g1, g2, gz, a % P1, (a / P1) % P2, a / (P1 * P2), Gv, w);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) G[g * gs + k * nlocp + a] = Gv[k];
    if (a == 0) W[g] = g < ng ? w : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, li = lane & 15, kk = lane >> 4;
  int I, J;
  std_pair(tiles, __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), I, J);
  double old[4][9];  // the direct block's CSR values, read now, added after the products
  std_add_early(d, vals, e1, e2, zsp, I, J, old);
  std_dbl4 m[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) m[e] = std_dbl4{0.0, 0.0, 0.0, 0.0};
  for (int st = 0; st < nsteps; ++st) {
    const int g = 4 * st + kk;
    const double *Gg = G + g * gs;
    const double w = W[g];
    double A[3], B[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      A[k] = w * Gg[k * nlocp + 16 * I + li];
      B[k] = Gg[k * nlocp + 16 * J + li];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) m[3 * k + l] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[k], B[l], m[3 * k + l], 0, 0, 0);
  }
  double ke[4][9];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int e = 0; e < 9; ++e) ke[v][e] = 0.0;
  std_contract(m, d.Eply + 81 * d.zply[c], ke);
  std_add_late(d, vals, e1, e2, zsp, I, J, ke, old);
}

// Elements of any number of ply cells: every (element, tile pair) is a
// wavefront of its own, the operands evaluated in the lanes from the basis
// tables and the element matrix summed over the span's cells in registers.
// For elements through many plies (the matrix costs far more than its
// read-modify-write) and for tables larger than the LDS.
__global__ void __launch_bounds__(64 * STD_WAVES, 2) k_std3d(Dev d, double *__restrict__ vals, int c1, int c2, int c3,
                                                             int n1c, int n2c, int64_t n_elem, int tiles) {
  const int units = tiles * (tiles + 1) / 2;
  // the wavefront's index, made explicitly uniform so the element's indices live in scalar registers
  const int64_t wid = std_block() * STD_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (wid >= n_elem * units) return;  // a whole wavefront; the kernel has no barrier
  const int64_t el = wid / units;
  int I, J, e1, e2, zsp;
  std_pair(tiles, (int)(wid - el * units), I, J);
  std_element(d, el, c1, c2, c3, n1c, n2c, e1, e2, zsp);
  const int lane = threadIdx.x & 63, li = lane & 15, kk = lane >> 4;
  const int P1 = d.p1 + 1, P2 = d.p2 + 1, Q1 = d.q + 1;
  const int nloc = P1 * P2 * Q1, ng = d.ng1 * d.ng2 * d.ngz, nsteps = (ng + 3) / 4;
  // this lane's operand functions (clamped to function 0 when padded: finite, then zeroed)
  const int ia = 16 * I + li, ib = 16 * J + li;
  const bool va = ia < nloc, vb = ib < nloc;
  const int ja = va ? ia : 0, jb = vb ? ib : 0;
  const int a1 = ja % P1, a2 = (ja / P1) % P2, at = ja / (P1 * P2);
  const int b1 = jb % P1, b2 = (jb / P1) % P2, bt = jb / (P1 * P2);
  double ke[4][9];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int e = 0; e < 9; ++e) ke[v][e] = 0.0;
  for (int ci = d.zs_cptr[zsp]; ci < d.zs_cptr[zsp + 1]; ++ci) {
    const int c = d.zs_cell[ci];
    std_dbl4 m[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = std_dbl4{0.0, 0.0, 0.0, 0.0};
    for (int st = 0; st < nsteps; ++st) {
      // A_k = w G_a(g)_k, B_l = G_b(g)_l at g = 4 st + kk (zero past the last point or function)
      const int g = 4 * st + kk;
      const bool vg = g < ng;
      const int gg = vg ? g : 0;
      const int g1 = gg % d.ng1, g2 = (gg / d.ng1) % d.ng2, gz = gg / (d.ng1 * d.ng2);
      double Ga[3], Gb[3], w, wb;
      std_gradient(d, e1, e2, c, g1, g2, gz, a1, a2, at, Ga, w);
      std_gradient(d, e1, e2, c, g1, g2, gz, b1, b2, bt, Gb, wb);
      const double sa = (va && vg) ? w : 0.0, sb = (vb && vg) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double A = sa * Ga[k];
#pragma unroll
        for (int l = 0; l < 3; ++l) m[3 * k + l] = __builtin_amdgcn_mfma_f64_16x16x4f64(A, sb * Gb[l], m[3 * k + l], 0, 0, 0);
      }
    }
    std_contract(m, d.Eply + 81 * d.zply[c], ke);
  }
  std_add(d, vals, e1, e2, zsp, I, J, ke);
}

// ---------------------------------------------------------------------------
// Adjoint.  K is linear in every ply's rotated tensor D_l (eq. Km_0); with the
// split of Sec. 3 written per ply, K = sum_l sum_ab Q_{l,ab} (x) P_ab[D_l] and
// P_ab[D][k][rt] = sum_kl M_ab[k][kl] E[D][kl][rt] (moments M of k_p2d,
// bracket coefficients E of D), so for L = <G, vals>
//   dL/dE_l[kl][rt] = Y_l[kl][rt] = sum_k sum_ab M_ab[k][kl] Z_{l,ab}[k][rt],
//   Z_{l,ab}[k][rt] = sum_zk Q_{l,ab}[zk] G[zk, k, r, t],
// and dL/dD_l[I][J] sums Y_l over the (k,r) with Voigt index I and (l,t) with J.
// dK is never formed: G is streamed once in the scatter's order.

// Per-ply 1D operators by accumulator slot (ply & 1), padded per thickness
// row to its longest width lz = 2q + 1: Qp[it][a][slot][ab] for the pair
// (it, a-th nonzero of row it), zeros for a past the row's width.
__global__ void k_q1d_ply(Dev d, int lz) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * (int64_t)d.nt * lz) return;
  const int slot = (int)(idx & 1), a = (int)((idx >> 1) % lz), it = (int)((idx >> 1) / lz);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int zk = d.zrow[it] + a;
  const bool in_row = zk < d.zrow[it + 1];
  const int jt = in_row ? d.zcol[zk] : 0, Q1 = d.q + 1;
  for (int ci = in_row ? d.zcptr[zk] : 0; ci < (in_row ? d.zcptr[zk + 1] : 0); ++ci) {
    const int c = d.zcell[ci];
    if ((d.zply[c] & 1) != slot) continue;
    const int ai = it - d.zfirst[c], aj = jt - d.zfirst[c];
    for (int g = 0; g < d.ngz; ++g) {
      const double *t = d.ztab + ((int64_t)c * d.ngz + g) * Q1 * 2;
      const double Ti = t[2 * ai], dTi = t[2 * ai + 1], Tj = t[2 * aj], dTj = t[2 * aj + 1];
      const double w = d.zw[(int64_t)c * d.ngz + g];
      acc[0] += w * Ti * Tj;
      acc[1] += w * Ti * dTj;
      acc[2] += w * dTi * Tj;
      acc[3] += w * dTi * dTj;
    }
  }
  double *o = d.Qp + 4 * idx;
  o[0] = acc[0];
  o[1] = acc[1];
  o[2] = acc[2];
  o[3] = acc[3];
}

// One block per scatter tile (whole in-plane rows), one thread per
// (in-plane nonzero k, component t).  Thickness rows are streamed in order
// (the next row's loads issued before the current row is used);
// Z of the (at most two) plies a row touches accumulates in registers; when
// a ply's last row is done the block contracts Z with its moments and sums
// over its nonzeros in LDS: adj_part[ply][kl][rt][tile].
constexpr int ADJ_THREADS = 256;

// Workgroup barrier that orders LDS accesses only: loads from global memory
// issued before it stay in flight (__syncthreads also waits for them, which
// would drain the stream's prefetch at every ply end).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LZ: the longest thickness row, 2q + 1.  RANK1: G = u u^T on the pattern
// (L = u^T K u), formed from u on the fly instead of read; src is u (n_rows
// doubles) then, else G (nnz doubles).
template <int LZ, bool RANK1>
__global__ void __launch_bounds__(ADJ_THREADS) k_adj_stream(Dev d, const double *__restrict__ src,
                                                            const double *__restrict__ qp) {
  __shared__ double red[ADJ_THREADS * 27];
  const int tile = blockIdx.x;
  const int k0 = d.tiles[tile], tk = d.tiles[tile + 1] - k0;
  const int sig = threadIdx.x;
  const bool act = sig < 3 * tk;
  const int kk = act ? sig / 3 : 0, t = act ? sig - 3 * kk : 0, k = k0 + kk;
  const int is = d.krow[k], sr = d.srow[is];
  const int Ls = d.srow[is + 1] - sr, off = 3 * (k - sr) + t;
  double m[4][9];
#pragma unroll
  for (int ab = 0; ab < 4; ++ab)
#pragma unroll
    for (int kl = 0; kl < 9; ++kl) {
      const double v = d.M[m_index(k, ab * 9 + kl)];  // k is valid for every thread
      m[ab][kl] = act ? v : 0.0;
    }
  double z[2][4][3];
#pragma unroll
  for (int sl = 0; sl < 2; ++sl)
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) z[sl][ab][0] = z[sl][ab][1] = z[sl][ab][2] = 0.0;
  const int64_t astride = 3 * (int64_t)Ls;
  // software pipeline over row pairs: the G values of the next row are in
  // flight while a row is contracted (one row's loads alone leave the stream
  // latency bound).  Every load is unconditional (rows past the last reload
  // it, never used): a load on only one path would make the wait for the
  // current row also wait for the next row's loads.  Inactive threads load
  // their block's first nonzero (in bounds), so the loads need no divergent
  // branch either.  RANK1 keeps the raw u values (u of the row's columns in
  // g[a][0], of the row itself in g[0][1], g[0][2], g[1][1]) and multiplies
  // when the row is used.
  const int js = d.kcol[k];
  auto load_row = [&](int it, double (&g)[LZ][3]) {
    it = it < d.nt ? it : d.nt - 1;
    const int zb = d.zrow[it], Lz = d.zrow[it + 1] - zb;
    if constexpr (RANK1) {
      // G[(it, is, r), (jt, js, t)] = u[3 (it ns + is) + r] u[3 (jt ns + js) + t]
      const double *ur = src + 3 * ((int64_t)it * d.ns + is);
      g[0][1] = ur[0];
      g[0][2] = ur[1];
      g[1][1] = ur[2];
#pragma unroll
      for (int a = 0; a < LZ; ++a) {
        const int ac = a < Lz ? a : Lz - 1;  // past the row: a valid address, weighted by 0
        g[a][0] = src[3 * ((int64_t)d.zcol[zb + ac] * d.ns + js) + t];
      }
    } else {
      const double *row = src + 9 * d.nnz2 * (int64_t)zb + 9 * (int64_t)Lz * sr + off;
      const int64_t rstride = 3 * (int64_t)Lz * Ls;
#pragma unroll
      for (int a = 0; a < LZ; ++a) {
        const int64_t ac = a < Lz ? a : Lz - 1;  // past the row: a valid address, weighted by 0
        g[a][0] = row[ac * astride];
        g[a][1] = row[rstride + ac * astride];
        g[a][2] = row[2 * rstride + ac * astride];
      }
    }
  };
  auto use_row = [&](int it, const double (&gin)[LZ][3]) {
    double g[LZ][3];
#pragma unroll
    for (int a = 0; a < LZ; ++a) {
      if constexpr (RANK1) {
        g[a][0] = gin[0][1] * gin[a][0];
        g[a][1] = gin[0][2] * gin[a][0];
        g[a][2] = gin[1][1] * gin[a][0];
      } else {
        g[a][0] = gin[a][0];
        g[a][1] = gin[a][1];
        g[a][2] = gin[a][2];
      }
    }
    const double *q = qp + (int64_t)it * LZ * 8;  // padded: zeros past the row's width
#pragma unroll
    for (int a = 0; a < LZ; ++a)
#pragma unroll
      for (int sl = 0; sl < 2; ++sl)
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) {
          const double qq = q[8 * a + 4 * sl + ab];
          z[sl][ab][0] += qq * g[a][0];
          z[sl][ab][1] += qq * g[a][1];
          z[sl][ab][2] += qq * g[a][2];
        }
    const int fin = d.rowfin[it];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      if (!(fin & (1 << sl))) continue;
      const int ply = d.rowply[2 * it + sl];
      // Y[kl][r] for this thread's t, into LDS
#pragma unroll
      for (int kl = 0; kl < 9; ++kl)
#pragma unroll
        for (int r = 0; r < 3; ++r)
          red[sig * 27 + kl * 3 + r] =
              m[0][kl] * z[sl][0][r] + m[1][kl] * z[sl][1][r] + m[2][kl] * z[sl][2][r] + m[3][kl] * z[sl][3][r];
#pragma unroll
      for (int ab = 0; ab < 4; ++ab) z[sl][ab][0] = z[sl][ab][1] = z[sl][ab][2] = 0.0;
      lds_barrier();
      if (sig < 81) {
        const int kl = sig / 9, r = (sig / 3) % 3, tt = sig % 3;
        double acc = 0.0;
        for (int q2 = 0; q2 < tk; ++q2) acc += red[(3 * q2 + tt) * 27 + kl * 3 + r];
        d.adj_part[((int64_t)ply * 81 + sig) * d.n_tiles + tile] = acc;
      }
      lds_barrier();
    }
  };
  double ga[LZ][3], gb[LZ][3];
  load_row(0, ga);
  for (int it = 0; it < d.nt; it += 2) {
    load_row(it + 1, gb);
    use_row(it, ga);
    load_row(it + 2, ga);
    if (it + 1 < d.nt) use_row(it + 1, gb);
  }
}

// Sum over the tiles of the partials of one (ply, entry) per block
// (adj_part[ply][81][tile]): each thread a strided run of tiles, then a tree,
// so the order is fixed and the result deterministic.
__global__ void __launch_bounds__(256) k_adj_reduce(Dev d) {
  __shared__ double part[256];
  const int idx = blockIdx.x;  // ply * 81 + entry
  const double *src = d.adj_part + (int64_t)idx * d.n_tiles;
  double acc = 0.0;
  for (int t = threadIdx.x; t < d.n_tiles; t += 256) acc += src[t];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) d.adj_y[idx] = part[0];
}

__device__ inline int voigt_pair(int i, int j) {
  if (i == j) return i;
  const int a = i < j ? i : j, b = i < j ? j : i;
  return a == 0 ? (b == 1 ? 3 : 4) : 5;
}

// Entries of the in-plane rotation R(theta) and of dR/dtheta as functions of
// their indices (no array indexed per thread); the Voigt stress transformation
// and its theta derivative follow by the product rule on its two R factors.
__device__ inline double rot_entry(int i, int k, double c, double s) {
  return i == 2 || k == 2 ? (i == k ? 1.0 : 0.0) : (i == k ? c : (i == 0 ? -s : s));
}
__device__ inline double drot_entry(int i, int k, double c, double s) {
  return i == 2 || k == 2 ? 0.0 : (i == k ? -s : (i == 0 ? -c : c));
}

// Per ply, one block (thread e < 36 owns the Voigt pair (I, J) = (e / 6, e % 6)):
// dL/dD_l[I][J] sums the entries of Y_l whose index pairs map to (I, J);
// dL/dtheta_l = <dL/dD_l, dT C T^T + T C dT^T> (a fixed-order sum over the 36
// products); and the ply's share T_l^T dL/dD_l T_l of its material's gradient,
// stored for k_adj_mat.
__global__ void __launch_bounds__(64) k_adj_ply(Dev d, const double *__restrict__ C, const double *__restrict__ theta,
                                                double *__restrict__ grad_theta) {
  __shared__ double sT[36], sdT[36], sD[36], sW[36], sp[36];
  const int l = blockIdx.x, e = threadIdx.x;
  const int I = e / 6, J = e - 6 * (e / 6);
  if (e < 36) {
    const double c = cos(theta[l]), s = sin(theta[l]);
    const int i = kVi[I], j = kVj[I], k = kVi[J], m = kVj[J];
    double t = rot_entry(i, k, c, s) * rot_entry(j, m, c, s);
    double dt = drot_entry(i, k, c, s) * rot_entry(j, m, c, s) + rot_entry(i, k, c, s) * drot_entry(j, m, c, s);
    if (k != m) {
      t += rot_entry(i, m, c, s) * rot_entry(j, k, c, s);
      dt += drot_entry(i, m, c, s) * rot_entry(j, k, c, s) + rot_entry(i, m, c, s) * drot_entry(j, k, c, s);
    }
    sT[e] = t;
    sdT[e] = dt;
    const double *Y = d.adj_y + 81 * l;
    double a = 0.0;
    for (int kk = 0; kk < 3; ++kk)
      for (int mm = 0; mm < 3; ++mm)
        for (int r = 0; r < 3; ++r)
          for (int tt = 0; tt < 3; ++tt)
            if (voigt_pair(kk, r) == I && voigt_pair(mm, tt) == J) a += Y[(kk * 3 + mm) * 9 + r * 3 + tt];
    sD[e] = a;
  }
  __syncthreads();
  if (e < 36) {
    const double *Cm = C + 36 * d.ply_mat[l];
    double a = 0.0;
    for (int K = 0; K < 6; ++K)
      for (int L = 0; L < 6; ++L) a += (sdT[6 * I + K] * sT[6 * J + L] + sT[6 * I + K] * sdT[6 * J + L]) * Cm[K * 6 + L];
    sp[e] = sD[e] * a;
    double w = 0.0;  // (dL/dD T)[I][J]
    for (int K = 0; K < 6; ++K) w += sD[6 * I + K] * sT[6 * K + J];
    sW[e] = w;
  }
  __syncthreads();
  if (e == 0) {
    double g = 0.0;
    for (int q = 0; q < 36; ++q) g += sp[q];
    grad_theta[l] = g;
  }
  if (e < 36) {  // (T^T dL/dD T)[A][B] with (A, B) = (I, J)
    double cm = 0.0;
    for (int K = 0; K < 6; ++K) cm += sT[6 * K + I] * sW[6 * K + J];
    d.adj_cm[36 * (int64_t)l + e] = cm;
  }
}

// dL/dC_m[A][B] = sum over the plies of material m (in order) of their shares.
__global__ void k_adj_mat(Dev d, double *__restrict__ grad_C) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 36 * d.n_mat) return;
  const int mt = idx / 36, e = idx - 36 * mt;
  double acc = 0.0;
  for (int l = 0; l < d.n_ply; ++l)
    if (d.ply_mat[l] == mt) acc += d.adj_cm[36 * (int64_t)l + e];
  grad_C[idx] = acc;
}

__global__ void k_rowptr(Dev d, int64_t *__restrict__ rowptr) {
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row > d.nrows) return;
  if (row == d.nrows) {
    rowptr[row] = d.nnz;
    return;
  }
  const int64_t i = row / 3;
  const int r = (int)(row % 3);
  const int it = (int)(i / d.ns), is = (int)(i % d.ns);
  const int zb = d.zrow[it], Lz = d.zrow[it + 1] - zb;
  const int sr = d.srow[is], Ls = d.srow[is + 1] - sr;
  rowptr[row] = 9 * d.nnz2 * (int64_t)zb + 3 * (int64_t)Lz * (3 * (int64_t)sr + (int64_t)r * Ls);
}

__global__ void __launch_bounds__(KRON_THREADS) k_colind(Dev d, int32_t *__restrict__ colind) {
  int tile, g;
  if (!kron_block(d, tile, g)) return;
  const int k0 = d.tiles[tile], tk = d.tiles[tile + 1] - k0;
  const int it0 = d.chunk_ptr[d.group_ptr[g]], it1 = d.chunk_ptr[d.group_ptr[g + 1]];
  for (int sig = threadIdx.x; sig < 3 * tk; sig += KRON_THREADS) {
    const int kk = sig / 3, t = sig - 3 * kk, k = k0 + kk;
    const int is = d.krow[k], js = d.kcol[k];
    const int sr = d.srow[is], Ls = d.srow[is + 1] - sr;
    for (int it = it0; it < it1; ++it) {
      const int zb = d.zrow[it], Lz = d.zrow[it + 1] - zb;
      int32_t *out = colind + 9 * d.nnz2 * (int64_t)zb + 9 * (int64_t)Lz * sr + 3 * (k - sr) + t;
      for (int a = 0; a < Lz; ++a) {
        const int32_t col = 3 * (d.zcol[zb + a] * d.ns + js) + t;
        for (int r = 0; r < 3; ++r) out[r * 3 * (int64_t)Lz * Ls + (int64_t)a * 3 * Ls] = col;
      }
    }
  }
}

lam_status hip_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? LAM_OK : LAM_EHIP;
}

int kron_grid(const lam_plan *p) {
  int nblk = p->n_tiles * p->n_groups;
  return 8 * ((nblk + 7) / 8);
}

void launch_kron(const lam_plan *p, const Dev &d, double *vals, hipStream_t s) {
  const int grid = kron_grid(p);
  const size_t lds = (size_t)p->kron_lds;
  const dim3 blk(p->kron_threads);
  switch (p->kron_nsc) {
    case 1:
      if (p->mat_field)
        hipLaunchKernelGGL((k_kron_reg<1, true>), dim3(grid), blk, lds, s, d, d.Qc, vals);
      else
        hipLaunchKernelGGL((k_kron_reg<1, false>), dim3(grid), blk, lds, s, d, d.Qc, vals);
      return;
    case 2:
      if (p->mat_field)
        hipLaunchKernelGGL((k_kron_reg<2, true>), dim3(grid), blk, lds, s, d, d.Qc, vals);
      else
        hipLaunchKernelGGL((k_kron_reg<2, false>), dim3(grid), blk, lds, s, d, d.Qc, vals);
      return;
    case 4: hipLaunchKernelGGL((k_kron_reg<4, false>), dim3(grid), blk, lds, s, d, d.Qc, vals); return;
    case 8: hipLaunchKernelGGL((k_kron_reg<8, false>), dim3(grid), blk, lds, s, d, d.Qc, vals); return;
    default: break;
  }
  if (p->chunk_sets > 0)
    hipLaunchKernelGGL((k_kron_lds<true>), dim3(grid), dim3(KRON_THREADS), lds, s, d, vals);
  else
    hipLaunchKernelGGL((k_kron_lds<false>), dim3(grid), dim3(KRON_THREADS), lds, s, d, vals);
}

lam_status check_ws(const lam_plan *p, const void *ws, int64_t ws_bytes) {
  if (!p || !ws) return LAM_EINVAL;
  if (ws_bytes < p->L.total) return LAM_ESIZE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return LAM_EINVAL;
  return LAM_OK;
}

}  // namespace

extern "C" LAM_API lam_status lam_plan_upload(const lam_plan *p, void *ws, int64_t ws_bytes, void *stream) {
  lam_status st = check_ws(p, ws, ws_bytes);
  if (st != LAM_OK) return st;
  hipError_t e = hipMemcpyAsync(ws, p->image.data(), p->L.const_bytes, hipMemcpyHostToDevice,
                                static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAM_OK : LAM_EHIP;
}

extern "C" LAM_API lam_status lam_check(const lam_plan *p, void *ws, int64_t ws_bytes, int32_t *flags, void *stream) {
  lam_status st = check_ws(p, ws, ws_bytes);
  if (st != LAM_OK) return st;
  if (!flags) return LAM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t *dev = at<int32_t>(ws, p->L.status);
  int32_t host[lam::N_STATUS];
  static const int32_t zeros[lam::N_STATUS] = {};
  if (hipMemcpyAsync(host, dev, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(dev, zeros, sizeof(zeros), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LAM_EHIP;
  *flags = (host[0] ? LAM_CHECK_BUCKET_ANGLES : 0) | (host[1] ? LAM_CHECK_HARMONIC5_COUPLING : 0);
  return LAM_OK;
}

extern "C" LAM_API lam_status lam_pattern(const lam_plan *p, const void *ws, int64_t ws_bytes, int64_t *rowptr,
                                          int32_t *colind, void *stream) {
  lam_status st = check_ws(p, ws, ws_bytes);
  if (st != LAM_OK) return st;
  if (!rowptr || !colind) return LAM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d = make_dev(p, const_cast<void *>(ws));
  int64_t nb = (p->nrows + 1 + 255) / 256;
  hipLaunchKernelGGL(k_rowptr, dim3((unsigned)nb), dim3(256), 0, s, d, rowptr);
  hipLaunchKernelGGL(k_colind, dim3(kron_grid(p)), dim3(KRON_THREADS), 0, s, d, colind);
  return hip_status();
}

namespace {

// The launches of the fast assembly (Sec. 3) on the device view d.
// Material fields: the rotated field at the in-plane Gauss points, P of every
// set integrated element by element with the field inside (one launch per
// element colour: elements of a colour share no in-plane function), and the
// 1D coefficients.  The scatter and the matrix-free product read P.
void launch_prep_field(const lam_plan *p, const Dev &d, const double *C, const double *theta, hipStream_t s) {
  const int64_t nq = p->nnzz * (p->kron_nsc > 0 ? p->kron_nsc : p->maxact);
  const int64_t npts = (int64_t)p->ne1 * p->ne2 * p->ng1 * p->ng2;
  hipLaunchKernelGGL(k_rotate_field, dim3((unsigned)(((int64_t)p->n_sets * p->ns + 255) / 256)), dim3(256), 0, s, d,
                     C, theta);
  hipLaunchKernelGGL(k_field_points, dim3((unsigned)((81 * npts * p->n_sets + 255) / 256)), dim3(256), 0, s, d);
  const int P1 = p->p1 + 1, P2 = p->p2 + 1, nb = P1 * P2, ngp = p->ng1 * p->ng2;
  const size_t lds = sizeof(double) * (size_t)ngp * (10 + 3 * nb + 81);
  const int thr = std::min(256, (nb * nb + 63) / 64 * 64);
  hipLaunchKernelGGL(k_fill_zero, dim3(2048), dim3(256), 0, s, d.P, (int64_t)p->n_sets * 36 * p->nnz2);
  for (int c2 = 0; c2 < P2; ++c2)
    for (int c1 = 0; c1 < P1; ++c1) {
      const int n1c = (p->ne1 - c1 + P1 - 1) / P1, n2c = (p->ne2 - c2 + P2 - 1) / P2;
      const int64_t nblk = (int64_t)n1c * n2c * p->n_sets;
      if (nblk > 0) hipLaunchKernelGGL(k_p2d_field, dim3((unsigned)nblk), dim3(thr), lds, s, d, c1, c2, n1c, n2c);
    }
  hipLaunchKernelGGL(k_q1d, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, d, theta);
}

void launch_assemble(const lam_plan *p, const Dev &d, const double *C, const double *theta, double *vals,
                     void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t nq = p->nnzz * (p->kron_nsc > 0 ? p->kron_nsc : p->maxact);
  if (p->mat_field) {
    launch_prep_field(p, d, C, theta, s);
    void *prof = lam::profile_begin(0, stream);
    launch_kron(p, d, vals, s);
    lam::profile_end(prof, stream);
    return;
  }
  hipLaunchKernelGGL(k_rotate, dim3((std::max(p->n_sets, p->n_ply) + 63) / 64), dim3(64), 0, s, d, C, theta);
  if (p->harm_ply) hipLaunchKernelGGL(k_harm_ply, dim3((p->n_ply + 63) / 64), dim3(64), 0, s, d, theta);
  if (p->kron_nsc > 0) {
    // register-mode scatter contracts P itself from the moments: one launch
    // for the moments and the 1D coefficients
    const int nb_m = (int)((p->nnz2 + 255) / 256), nb_q = (int)((nq + 3) / 4);
    hipLaunchKernelGGL(k_prep, dim3((unsigned)(nb_m + nb_q)), dim3(256), 0, s, d, theta, nb_m);
  } else {
    // LDS mode reads P, which needs the set tensors
    hipLaunchKernelGGL(k_p2d, dim3((unsigned)((p->nnz2 + 255) / 256)), dim3(256), 0, s, d, d.Ec, d.P, d.M, 1);
    hipLaunchKernelGGL(k_q1d, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, d, theta);
  }
  void *prof = lam::profile_begin(0, stream);
  launch_kron(p, d, vals, s);
  lam::profile_end(prof, stream);
}

}  // namespace

// Static scratch of lam_assemble_static: one copy per GPU for the life of the
// process, shared by every call on that GPU.  Host code never uses the
// array's name as an address: each device's copy is looked up once with
// hipGetSymbolAddress (with that device current) and kept in scratch_dev.
constexpr int64_t STATIC_SCRATCH_BYTES = int64_t(LAM_STATIC_SCRATCH_MIB) << 20;
static __device__ __align__(256) double scratch[STATIC_SCRATCH_BYTES / 8];

namespace {

constexpr int MAX_DEVICES = 64;
void *scratch_dev[MAX_DEVICES];
std::mutex scratch_mu;

// The calling thread's current device's copy of scratch, or null on a HIP error.
void *static_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    scratch_dev[dev] = ptr;
  }
  return scratch_dev[dev];
}

}  // namespace

extern "C" LAM_API lam_status lam_assemble(const lam_plan *p, void *ws, int64_t ws_bytes, const double *C,
                                           const double *theta, double *vals, int64_t nnz, void *stream) {
  lam_status st = check_ws(p, ws, ws_bytes);
  if (st != LAM_OK) return st;
  if (!C || !theta || !vals) return LAM_EINVAL;
  if (nnz != p->nnz) return LAM_ESIZE;
  launch_assemble(p, make_dev(p, ws), C, theta, vals, stream);
  return hip_status();
}

extern "C" LAM_API lam_status lam_assemble_static(const lam_plan *p, void *ws, int64_t ws_bytes, const double *C,
                                                  const double *theta, double *vals, int64_t nnz, void *stream) {
  if (!p || !ws || !C || !theta || !vals) return LAM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return LAM_EINVAL;
  if (ws_bytes < p->L.const_bytes || nnz != p->nnz) return LAM_ESIZE;
  if (p->L.fwd_end - p->L.const_bytes > STATIC_SCRATCH_BYTES) return LAM_ESCRATCH;
  void *sbase = static_scratch();
  if (!sbase) return LAM_EHIP;
  launch_assemble(p, make_dev(p, ws, sbase), C, theta, vals, stream);
  return hip_status();
}

namespace {

// The set tensors and the moments and 1D coefficients the register-mode
// scatter and the matrix-free product read.
void launch_prep(const lam_plan *p, const Dev &d, const double *C, const double *theta, hipStream_t s) {
  if (p->mat_field) {
    launch_prep_field(p, d, C, theta, s);
    return;
  }
  const int64_t nq = p->nnzz * p->kron_nsc;
  const int nb_m = (int)((p->nnz2 + 255) / 256), nb_q = (int)((nq + 3) / 4);
  hipLaunchKernelGGL(k_rotate, dim3((std::max(p->n_sets, p->n_ply) + 63) / 64), dim3(64), 0, s, d, C, theta);
  if (p->harm_ply) hipLaunchKernelGGL(k_harm_ply, dim3((p->n_ply + 63) / 64), dim3(64), 0, s, d, theta);
  hipLaunchKernelGGL(k_prep, dim3((unsigned)(nb_m + nb_q)), dim3(256), 0, s, d, theta, nb_m);
}

void launch_apply(const lam_plan *p, const Dev &d, const double *u, const uint8_t *fixed, double *y, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t lds = (size_t)(p->kron_lds + APPLY_ROWS * 3 * sizeof(double) * 3 * p->tile_k);
  void *prof = lam::profile_begin(4, stream);
  const dim3 grid(kron_grid(p)), blk(p->kron_threads);
  if (p->kron_nsc == 1 && p->mat_field)
    hipLaunchKernelGGL((k_apply<1, true>), grid, blk, lds, s, d, d.Qc, u, fixed, y);
  else if (p->kron_nsc == 1)
    hipLaunchKernelGGL((k_apply<1, false>), grid, blk, lds, s, d, d.Qc, u, fixed, y);
  else if (p->mat_field)
    hipLaunchKernelGGL((k_apply<2, true>), grid, blk, lds, s, d, d.Qc, u, fixed, y);
  else
    hipLaunchKernelGGL((k_apply<2, false>), grid, blk, lds, s, d, d.Qc, u, fixed, y);
  lam::profile_end(prof, stream);
}

}  // namespace

extern "C" LAM_API lam_status lam_apply(const lam_plan *p, void *ws, int64_t ws_bytes, const double *C,
                                        const double *theta, const double *u, const uint8_t *fixed,
                                        int64_t n_rows, double *y, void *stream) {
  lam_status st = check_ws(p, ws, ws_bytes);
  if (st != LAM_OK) return st;
  if (!C || !theta || !u || !y) return LAM_EINVAL;
  if (n_rows != p->nrows) return LAM_ESIZE;
  if (p->kron_nsc < 1 || p->kron_nsc > 2) return LAM_EUNSUP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d = make_dev(p, ws);
  launch_prep(p, d, C, theta, s);
  launch_apply(p, d, u, fixed, y, stream);
  return hip_status();
}

// ---------------------------------------------------------------------------
// Conjugate gradients on the Dirichlet-eliminated operator A = P K P + (I - P)
// (P: projection on the free rows) with right-hand side P b, so the fixed
// entries of the solution go to zero, preconditioned by thickness lines: for
// every in-plane function is, the block of A that couples all thickness
// functions and displacement components of is (3 nt unknowns, banded with
// half bandwidth 3q + 2), factored once by a banded Cholesky and solved at
// every iteration.  In a thin laminate the coupling through the thickness is
// the stiff one (plies much thinner than the in-plane elements), which a
// pointwise preconditioner leaves untouched.  Every vector operation is a
// kernel, the scalars stay on the device, the dot products are two-stage
// fixed-order sums (deterministic).  work (doubles): r, p, q = A p,
// z = M^{-1} r (n each), the line factors (ns * 3 nt * (3q + 3)), 2 CG_PARTS
// partial sums, 6 scalars {r.z, p.q, new r.z, P b . P b, r.r, spare}.
constexpr int CG_PARTS = 512;
// iterations between two host reads of the residual (each read waits for the
// stream); up to CG_CHECK - 1 iterations may run past the tolerance
constexpr int CG_CHECK = 8;

// Thickness line of in-plane function is: A's entries between (it, r) and
// (jt, t), from the split (eq. Km_2) at the in-plane diagonal nonzero k_d of
// is: sum over row it's set slots u and ab of Qc[(it, jt)][u][ab] P_u[k_d][ab][r][t],
// P_u = sum_kl M_ab[kl][k_d] E_u[kl] (the register-mode scatter's moments and
// brackets; with FIELD, material fields, the stored P of the slot's set).  Fixed components take a unit row and column.  The lower band
// (row i = 3 it + r, column i - c for c = 0..3q+2) is stored at
// fac[(i (3q + 3) + c) ns + is] (consecutive lines on consecutive addresses)
// and overwritten by its Cholesky factor.  One thread per line.
template <int NSC, bool FIELD>
__global__ void __launch_bounds__(256) k_cg_lines(Dev d, const double *__restrict__ qd,
                                                  const uint8_t *__restrict__ fixed, double *__restrict__ fac) {
  const int is = blockIdx.x * blockDim.x + threadIdx.x;
  if (is >= d.ns) return;
  const int hb = 3 * d.q + 2, wb = hb + 1, n = 3 * d.nt;
  const int64_t ns = d.ns;
  const int i1 = is % d.n1, i2 = is / d.n1;
  const int64_t k = d.srow[is] + (int64_t)(i2 - d.a2f[i2]) * d.a1c[i1] + (i1 - d.a1f[i1]);
  double mv[4][9];
  if constexpr (!FIELD) {
#pragma unroll
    for (int ab = 0; ab < 4; ++ab)
#pragma unroll
      for (int kl = 0; kl < 9; ++kl) mv[ab][kl] = d.M[m_index(k, ab * 9 + kl)];
  }
  for (int64_t e = 0; e < (int64_t)n * wb; ++e) fac[e * ns + is] = 0.0;
  for (int it = 0; it < d.nt; ++it) {
    const int ch = d.zchunk[it], c0 = d.chunk_sptr[ch], nsc = d.chunk_sptr[ch + 1] - c0;
    double pu[NSC][4][9];  // P of the row's slots at the diagonal in-plane nonzero
#pragma unroll
    for (int u = 0; u < NSC; ++u) {
      const int gs = u < nsc ? d.chunk_set[c0 + u] : d.chunk_set[c0];
      if constexpr (FIELD) {
#pragma unroll
        for (int ab = 0; ab < 4; ++ab)
#pragma unroll
          for (int rt = 0; rt < 9; ++rt)
            pu[u][ab][rt] = u < nsc ? d.P[((int64_t)gs * 36 + ab * 9 + rt) * d.nnz2 + k] : 0.0;
        continue;
      }
      const double *E = d.Escat + 81 * (int64_t)gs;
#pragma unroll
      for (int ab = 0; ab < 4; ++ab)
#pragma unroll
        for (int rt = 0; rt < 9; ++rt) {
          double a = 0.0;
#pragma unroll
          for (int kl = 0; kl < 9; ++kl) a += mv[ab][kl] * E[kl * 9 + rt];
          pu[u][ab][rt] = u < nsc ? a : 0.0;
        }
    }
    const int zb = d.zrow[it], Lz = d.zrow[it + 1] - zb;
    for (int x = 0; x < Lz; ++x) {
      const int jt = d.zcol[zb + x];
      if (jt > it) break;  // columns ascend: the rest is above the diagonal
      const double *q = qd + 4 * ((int64_t)(zb + x) * NSC);
      for (int r = 0; r < 3; ++r)
        for (int t = 0; t < 3; ++t) {
          const int i = 3 * it + r, j = 3 * jt + t;
          if (j > i) continue;
          double v = 0.0;
#pragma unroll
          for (int u = 0; u < NSC; ++u)
#pragma unroll
            for (int ab = 0; ab < 4; ++ab) v += q[4 * u + ab] * pu[u][ab][3 * r + t];
          const int64_t gi = 3 * ((int64_t)it * ns + is) + r, gj = 3 * ((int64_t)jt * ns + is) + t;
          if (fixed && (fixed[gi] || fixed[gj])) v = (i == j) ? 1.0 : 0.0;
          fac[((int64_t)i * wb + (i - j)) * ns + is] = v;
        }
    }
  }
  // banded Cholesky in place: L[i][j] at band column i - j
  for (int i = 0; i < n; ++i) {
    const int j0 = i - hb > 0 ? i - hb : 0;
    for (int j = j0; j <= i; ++j) {
      double sum = fac[((int64_t)i * wb + (i - j)) * ns + is];
      const int p0 = (i - hb > j - hb ? i - hb : j - hb) > 0 ? (i - hb > j - hb ? i - hb : j - hb) : 0;
      for (int pp = p0; pp < j; ++pp)
        sum -= fac[((int64_t)i * wb + (i - pp)) * ns + is] * fac[((int64_t)j * wb + (j - pp)) * ns + is];
      if (i == j)  // the diagonal slot keeps 1 / L_ii (SPD: sum > 0; the guard keeps it finite)
        fac[((int64_t)i * wb) * ns + is] = sum > 0.0 ? 1.0 / sqrt(sum) : 1.0;
      else
        fac[((int64_t)i * wb + (i - j)) * ns + is] = sum * fac[((int64_t)j * wb) * ns + is];
    }
  }
}

// z = M^{-1} r on every thickness line (forward and backward substitution
// with the banded factor, whose diagonal slots hold 1 / L_ii); with p given,
// p = z too.  One thread per line, one wavefront per block (the lines spread
// over as many compute units as there are wavefronts).  The substitutions are
// chains of dependent steps, so each step's operands (its factor row or
// column, its right-hand side) are loaded LS_AHEAD steps ahead into a ring of
// register slots: a step waits on loads issued LS_AHEAD steps before, not on
// its own.  The last HB = 3Q + 2 results stay in registers (a window shifted
// by one per step).
constexpr int LS_AHEAD = 5;

template <int Q>
__global__ void __launch_bounds__(64) k_cg_line_solve(Dev d, const double *__restrict__ fac,
                                                      const double *__restrict__ r, double *__restrict__ z,
                                                      double *__restrict__ p) {
  constexpr int HB = 3 * Q + 2, WB = HB + 1;
  const int is = blockIdx.x * blockDim.x + threadIdx.x;
  if (is >= d.ns) return;
  const int n = 3 * d.nt;
  const int64_t ns = d.ns;
  auto row = [&](int i) { return 3 * ((int64_t)(i / 3) * ns + is) + i % 3; };
  // slot: [0] 1 / L_ii, [c] the band entry at distance c (c = 1..HB), [WB] the right-hand side.
  // Loads past either end read the last (first) row instead (in bounds, never used), so the
  // loads carry no branch and the compiler keeps them in flight.
  double sl[LS_AHEAD][WB + 1];
  double win[HB];
  // L y = r (y kept in z); band entries before the first row are zero in the factor
  auto fwd_load = [&](int i, double *o) {
    const int ic = i < n ? i : n - 1;
    const double *Li = fac + (int64_t)ic * WB * ns + is;
#pragma unroll
    for (int c = 0; c <= HB; ++c) o[c] = Li[c * ns];
    o[WB] = r[row(ic)];
  };
  auto fwd_step = [&](int i, const double *o) {
    double sum = o[WB];
#pragma unroll
    for (int c = 1; c <= HB; ++c) sum -= o[c] * win[HB - c];
    const double y = sum * o[0];
#pragma unroll
    for (int c = 0; c + 1 < HB; ++c) win[c] = win[c + 1];
    win[HB - 1] = y;
    z[row(i)] = y;
  };
#pragma unroll
  for (int c = 0; c < HB; ++c) win[c] = 0.0;  // win[HB - c] = y[i - c] for c = 1..HB
#pragma unroll
  for (int j = 0; j < LS_AHEAD; ++j) fwd_load(j, sl[j]);
  const int nfull = n / LS_AHEAD * LS_AHEAD;
  for (int i0 = 0; i0 < nfull; i0 += LS_AHEAD) {
#pragma unroll
    for (int j = 0; j < LS_AHEAD; ++j) {
      fwd_step(i0 + j, sl[j]);
      fwd_load(i0 + j + LS_AHEAD, sl[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < LS_AHEAD; ++j)
    if (nfull + j < n) fwd_step(nfull + j, sl[j]);
  // L^T z = y: column i of L below the diagonal is L[i + c][c], c = 1..HB (zero past the last row)
  auto bwd_load = [&](int i, double *o) {
    const int ic = i >= 0 ? i : 0;
    o[0] = fac[(int64_t)ic * WB * ns + is];
#pragma unroll
    for (int c = 1; c <= HB; ++c) {
      const int rc = ic + c < n ? ic + c : n - 1;
      const double v = fac[((int64_t)rc * WB + c) * ns + is];
      o[c] = ic + c < n ? v : 0.0;
    }
    o[WB] = z[row(ic)];
  };
  auto bwd_step = [&](int i, const double *o) {
    double sum = o[WB];
#pragma unroll
    for (int c = 1; c <= HB; ++c) sum -= o[c] * win[c - 1];
    const double v = sum * o[0];
#pragma unroll
    for (int c = HB - 1; c > 0; --c) win[c] = win[c - 1];
    win[0] = v;
    z[row(i)] = v;
    if (p) p[row(i)] = v;
  };
#pragma unroll
  for (int c = 0; c < HB; ++c) win[c] = 0.0;  // win[c - 1] = z[i + c] for c = 1..HB
#pragma unroll
  for (int j = 0; j < LS_AHEAD; ++j) bwd_load(n - 1 - j, sl[j]);
  for (int i0 = n - 1; i0 >= n - nfull; i0 -= LS_AHEAD) {
#pragma unroll
    for (int j = 0; j < LS_AHEAD; ++j) {
      bwd_step(i0 - j, sl[j]);
      bwd_load(i0 - j - LS_AHEAD, sl[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < LS_AHEAD; ++j)
    if (n - 1 - nfull - j >= 0) bwd_step(n - 1 - nfull - j, sl[j]);
}

void launch_line_solve(const lam_plan *pl, const Dev &d, const double *fac, const double *r, double *z, double *pv,
                       hipStream_t s) {
  const dim3 lg((unsigned)((pl->ns + 63) / 64)), vb(64);
  switch (pl->q) {
    case 1: hipLaunchKernelGGL((k_cg_line_solve<1>), lg, vb, 0, s, d, fac, r, z, pv); break;
    case 2: hipLaunchKernelGGL((k_cg_line_solve<2>), lg, vb, 0, s, d, fac, r, z, pv); break;
    case 3: hipLaunchKernelGGL((k_cg_line_solve<3>), lg, vb, 0, s, d, fac, r, z, pv); break;
    default: hipLaunchKernelGGL((k_cg_line_solve<4>), lg, vb, 0, s, d, fac, r, z, pv); break;
  }
}

// partial sums of a.b (and, if c is given, of a.c) over blocks of a grid-stride loop
__global__ void __launch_bounds__(256) k_dot_partial(const double *__restrict__ a, const double *__restrict__ b,
                                                     const double *__restrict__ c, const uint8_t *__restrict__ fixed,
                                                     int64_t n, double *__restrict__ part) {
  __shared__ double sh[2][256];
  double ab = 0.0, ac = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    if (!(fixed && fixed[i])) {
      ab += a[i] * b[i];
      if (c) ac += a[i] * c[i];
    }
  sh[0][threadIdx.x] = ab;
  sh[1][threadIdx.x] = ac;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sh[0][0];
    part[CG_PARTS + blockIdx.x] = sh[1][0];
  }
}

// out[0] = sum of part[0..CG_PARTS), out[two] = sum of part[CG_PARTS..2 CG_PARTS) if two > 0
__global__ void __launch_bounds__(256) k_dot_final(const double *__restrict__ part, double *__restrict__ out, int two) {
  __shared__ double sh[2][256];
  sh[0][threadIdx.x] = part[threadIdx.x] + part[threadIdx.x + 256];
  sh[1][threadIdx.x] = part[CG_PARTS + threadIdx.x] + part[CG_PARTS + threadIdx.x + 256];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sh[0][0];
    if (two > 0) out[two] = sh[1][0];
  }
}

// r = P b - A x
__global__ void k_cg_init(int64_t n, const double *__restrict__ b, const double *__restrict__ ax,
                          const uint8_t *__restrict__ fixed, double *__restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  r[i] = (fixed && fixed[i] ? 0.0 : b[i]) - ax[i];
}

// alpha = (r.z) / (p.q); x += alpha p; r -= alpha q.  alpha = 0 once p.q is
// zero (p = 0: an iteration after the exact solution, see CG_CHECK)
__global__ void k_cg_step(int64_t n, const double *__restrict__ scal, const double *__restrict__ p,
                          const double *__restrict__ q, double *__restrict__ x, double *__restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double alpha = scal[1] != 0.0 ? scal[0] / scal[1] : 0.0;
  x[i] += alpha * p[i];
  r[i] -= alpha * q[i];
}

// beta = (new r.z) / (r.z); p = z + beta p (beta = 0 once r.z is zero)
__global__ void k_cg_dir(int64_t n, const double *__restrict__ scal, const double *__restrict__ z,
                         double *__restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = z[i] + (scal[0] != 0.0 ? scal[2] / scal[0] : 0.0) * p[i];
}

__global__ void k_scalar_copy(double *__restrict__ scal, int to, int from) {
  if (threadIdx.x == 0 && blockIdx.x == 0) scal[to] = scal[from];
}

namespace {

// out[0] = a.b (fixed rows skipped if fixed is given); with c, out[two] = a.c too
void launch_dot(const double *a, const double *b, const double *c, const uint8_t *fixed, int64_t n, double *part,
                double *out, int two, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(CG_PARTS), dim3(256), 0, s, a, b, c, fixed, n, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, part, out, two);
}

}  // namespace

namespace {

int64_t cg_factor_doubles(const lam_plan *p) { return (int64_t)p->ns * 3 * p->nt * (3 * p->q + 3); }

}  // namespace

extern "C" LAM_API int64_t lam_cg_work_bytes(const lam_plan *p) {
  return p ? (int64_t)sizeof(double) * (4 * p->nrows + cg_factor_doubles(p) + 2 * CG_PARTS + 6) : 0;
}

extern "C" LAM_API lam_status lam_cg(const lam_plan *p, void *ws, int64_t ws_bytes, const double *C,
                                     const double *theta, const uint8_t *fixed, const double *b, double *x,
                                     int64_t n_rows, void *work, int64_t work_bytes, double tol, int32_t max_iter,
                                     int32_t *iters, double *rel_res, void *stream) {
  lam_status st = check_ws(p, ws, ws_bytes);
  if (st != LAM_OK) return st;
  if (!C || !theta || !b || !x || !work || !iters || !rel_res || max_iter < 0 || !(tol >= 0.0)) return LAM_EINVAL;
  if (n_rows != p->nrows || work_bytes < lam_cg_work_bytes(p)) return LAM_ESIZE;
  if (p->kron_nsc < 1 || p->kron_nsc > 2) return LAM_EUNSUP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d = make_dev(p, ws);
  const int64_t n = n_rows;
  double *r = static_cast<double *>(work), *pv = r + n, *q = pv + n, *z = q + n, *fac = z + n;
  double *part = fac + cg_factor_doubles(p), *scal = part + 2 * CG_PARTS;
  const dim3 vg((unsigned)((n + 255) / 256)), lg((unsigned)((p->ns + 255) / 256)), vb(256);
  launch_prep(p, d, C, theta, s);
  if (p->kron_nsc == 1 && p->mat_field)
    hipLaunchKernelGGL((k_cg_lines<1, true>), lg, vb, 0, s, d, d.Qc, fixed, fac);
  else if (p->kron_nsc == 1)
    hipLaunchKernelGGL((k_cg_lines<1, false>), lg, vb, 0, s, d, d.Qc, fixed, fac);
  else if (p->mat_field)
    hipLaunchKernelGGL((k_cg_lines<2, true>), lg, vb, 0, s, d, d.Qc, fixed, fac);
  else
    hipLaunchKernelGGL((k_cg_lines<2, false>), lg, vb, 0, s, d, d.Qc, fixed, fac);
  launch_apply(p, d, x, fixed, q, stream);
  hipLaunchKernelGGL(k_cg_init, vg, vb, 0, s, n, b, q, fixed, r);
  launch_line_solve(p, d, fac, r, z, pv, s);
  launch_dot(b, b, nullptr, fixed, n, part, scal + 3, 0, s);
  launch_dot(r, z, r, nullptr, n, part, scal + 0, 4, s);  // r.z -> scal[0], r.r -> scal[4]
  double host[6];
  if (hipMemcpyAsync(host, scal, 6 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LAM_EHIP;
  const double bb = host[3];
  double rr = host[4];
  int it = 0;
  while (it < max_iter && !(bb > 0.0 ? rr <= tol * tol * bb : rr == 0.0)) {
    const int batch = max_iter - it < CG_CHECK ? max_iter - it : CG_CHECK;
    for (int k = 0; k < batch; ++k) {
      launch_apply(p, d, pv, fixed, q, stream);
      launch_dot(pv, q, nullptr, nullptr, n, part, scal + 1, 0, s);
      hipLaunchKernelGGL(k_cg_step, vg, vb, 0, s, n, scal, pv, q, x, r);
      launch_line_solve(p, d, fac, r, z, nullptr, s);
      launch_dot(r, z, r, nullptr, n, part, scal + 2, 2, s);  // new r.z -> scal[2], r.r -> scal[4]
      hipLaunchKernelGGL(k_cg_dir, vg, vb, 0, s, n, scal, z, pv);
      hipLaunchKernelGGL(k_scalar_copy, dim3(1), dim3(64), 0, s, scal, 0, 2);
    }
    if (hipMemcpyAsync(&rr, scal + 4, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return LAM_EHIP;
    it += batch;
  }
  *iters = it;
  *rel_res = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
  return hip_status();
}

extern "C" LAM_API lam_status lam_assemble_standard(const lam_plan *p, void *ws, int64_t ws_bytes, const double *C,
                                                    const double *theta, double *vals, int64_t nnz, void *stream) {
  lam_status st = check_ws(p, ws, ws_bytes);
  if (st != LAM_OK) return st;
  if (!C || !theta || !vals) return LAM_EINVAL;
  if (nnz != p->nnz) return LAM_ESIZE;
  const int P1 = p->p1 + 1, P2 = p->p2 + 1, Q1 = p->q + 1;
  const int nloc = P1 * P2 * Q1;
  if (p->mat_field) return LAM_EUNSUP;
  const int tiles = (nloc + 15) / 16, units = tiles * (tiles + 1) / 2;
  // one ply cell per element, at most eight tile pairs and a gradient table
  // within 80 KiB: the block-per-element kernel with the table in LDS
  const int nlocp = 16 * tiles, ngp = 4 * ((p->ng1 * p->ng2 * p->ngz + 3) / 4);
  const int gs = 3 * nlocp + ((3 * nlocp) % 32 == 0 ? 16 : 0);
  const size_t lds = sizeof(double) * ((size_t)ngp * gs + ngp);
  const bool use_lds = p->max_span_cells == 1 && units <= STD_LDS_WAVES && lds <= 80 * 1024;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d = make_dev(p, ws);
  hipLaunchKernelGGL(k_rotate_plies, dim3((p->n_ply + 63) / 64), dim3(64), 0, s, d, C, theta);
  void *prof_fill = lam::profile_begin(5, stream);
  hipLaunchKernelGGL(k_fill_zero, dim3(4096), dim3(256), 0, s, vals, p->nnz);
  lam::profile_end(prof_fill, stream);
  void *prof = lam::profile_begin(1, stream);
  for (int c3 = 0; c3 < Q1; ++c3)
    for (int c2 = 0; c2 < P2; ++c2)
      for (int c1 = 0; c1 < P1; ++c1) {
        const int n1c = (p->ne1 - c1 + P1 - 1) / P1, n2c = (p->ne2 - c2 + P2 - 1) / P2;
        const int n3c = (p->nzs - c3 + Q1 - 1) / Q1;
        const int64_t n = (int64_t)n1c * n2c * n3c;
        if (n <= 0) continue;
        if (use_lds) {
          hipLaunchKernelGGL(k_std3d_lds, dim3((unsigned)((n + 7) / 8 * 8)), dim3(64 * units), lds, s, d, vals, c1,
                             c2, c3, n1c, n2c, n, tiles, nlocp, gs);
        } else {
          const int64_t nb = ((n * units + STD_WAVES - 1) / STD_WAVES + 7) / 8 * 8;
          hipLaunchKernelGGL(k_std3d, dim3((unsigned)nb), dim3(64 * STD_WAVES), 0, s, d, vals, c1, c2, c3, n1c, n2c, n,
                             tiles);
        }
      }
  lam::profile_end(prof, stream);
  return hip_status();
}

namespace {

// The adjoint's launches; src is G (nnz doubles) or, rank1, u (n_rows doubles).
void launch_adjoint(const lam_plan *p, const Dev &d, const double *C, const double *theta, const double *src,
                    bool rank1, double *grad_C, double *grad_theta, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_p2d, dim3((unsigned)((p->nnz2 + 255) / 256)), dim3(256), 0, s, d, d.Ec, d.P, d.M, 0);
  const int lz = 2 * p->q + 1;
  hipLaunchKernelGGL(k_q1d_ply, dim3((unsigned)((2 * (int64_t)p->nt * lz + 255) / 256)), dim3(256), 0, s, d, lz);
  void *prof = lam::profile_begin(2, stream);
  const dim3 grid(p->n_tiles), blk(ADJ_THREADS);
  switch (p->q * 2 + (rank1 ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((k_adj_stream<3, false>), grid, blk, 0, s, d, src, d.Qp); break;
    case 3: hipLaunchKernelGGL((k_adj_stream<3, true>), grid, blk, 0, s, d, src, d.Qp); break;
    case 4: hipLaunchKernelGGL((k_adj_stream<5, false>), grid, blk, 0, s, d, src, d.Qp); break;
    case 5: hipLaunchKernelGGL((k_adj_stream<5, true>), grid, blk, 0, s, d, src, d.Qp); break;
    case 6: hipLaunchKernelGGL((k_adj_stream<7, false>), grid, blk, 0, s, d, src, d.Qp); break;
    case 7: hipLaunchKernelGGL((k_adj_stream<7, true>), grid, blk, 0, s, d, src, d.Qp); break;
    case 8: hipLaunchKernelGGL((k_adj_stream<9, false>), grid, blk, 0, s, d, src, d.Qp); break;
    default: hipLaunchKernelGGL((k_adj_stream<9, true>), grid, blk, 0, s, d, src, d.Qp); break;
  }
  lam::profile_end(prof, stream);
  hipLaunchKernelGGL(k_adj_reduce, dim3(81 * p->n_ply), dim3(256), 0, s, d);
  hipLaunchKernelGGL(k_adj_ply, dim3(p->n_ply), dim3(64), 0, s, d, C, theta, grad_theta);
  hipLaunchKernelGGL(k_adj_mat, dim3((36 * p->n_mat + 63) / 64), dim3(64), 0, s, d, grad_C);
}

}  // namespace

extern "C" LAM_API lam_status lam_adjoint(const lam_plan *p, void *ws, int64_t ws_bytes, const double *C,
                                          const double *theta, const double *grad_vals, int64_t nnz, double *grad_C,
                                          double *grad_theta, void *stream) {
  lam_status st = check_ws(p, ws, ws_bytes);
  if (st != LAM_OK) return st;
  if (!C || !theta || !grad_vals || !grad_C || !grad_theta) return LAM_EINVAL;
  if (nnz != p->nnz) return LAM_ESIZE;
  if (!p->adj_ok || 3 * p->tile_k > ADJ_THREADS) return LAM_EUNSUP;
  Dev d = make_dev(p, ws);
  launch_adjoint(p, d, C, theta, grad_vals, false, grad_C, grad_theta, stream);
  return hip_status();
}

extern "C" LAM_API lam_status lam_adjoint_rank1(const lam_plan *p, void *ws, int64_t ws_bytes, const double *C,
                                                const double *theta, const double *u, int64_t n_rows,
                                                double *grad_C, double *grad_theta, void *stream) {
  lam_status st = check_ws(p, ws, ws_bytes);
  if (st != LAM_OK) return st;
  if (!C || !theta || !u || !grad_C || !grad_theta) return LAM_EINVAL;
  if (n_rows != p->nrows) return LAM_ESIZE;
  if (!p->adj_ok || 3 * p->tile_k > ADJ_THREADS) return LAM_EUNSUP;
  Dev d = make_dev(p, ws);
  launch_adjoint(p, d, C, theta, u, true, grad_C, grad_theta, stream);
  return hip_status();
}
