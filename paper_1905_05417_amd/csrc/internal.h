// internal.h -- plan structure and workspace layout shared by the host plan
// (plan.cpp) and the device code (kernels.hip).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <vector>

#include "lamasm.h"

namespace lam {

constexpr int MAXP = 4;      // largest supported degree (in-plane and thickness)
constexpr int MAXG = 8;      // largest Gauss rule per direction
constexpr int NHARM_MAX = 9; // harmonics of D(theta) for a general 6x6
// status words of a workspace: [0] a bucket set's plies were given different
// angles, [1] a harmonic5 set's material couples {11,22,33,12} with {13,23}
constexpr int N_STATUS = 2;

// A byte range of the device workspace.
struct Region {
  int64_t off = 0, bytes = 0;
};

// Device workspace layout.  The "constant" part (tables) is written once by
// lam_plan_upload; the rest is scratch overwritten by every assembly.
struct Layout {
  // in-plane basis, per direction: tab[e][g][a] = (N, dN/dxi), w[e][g] = Gauss weight * half span
  Region tab1, w1, tab2, w2;
  // first function index of every in-plane element (knot span - degree)
  Region e1first, e2first;
  // per 1D overlap pair (i,j) of each direction: first shared element and count
  Region pe1, pe2;
  // in-plane pattern: srow[ns+1]; per in-plane nonzero k: row is, column js, 1D pair indices
  Region srow, krow, kcol, kp1, kp2;
  // thickness cells (ply x knot span): first function, ply, basis table, weights
  Region zfirst, zply, ztab, zw;
  // thickness pattern: zrow[nt+1], zcol[nnzz], zkrow[nnzz]; cells shared by each pair
  Region zrow, zcol, zkrow, zcptr, zcell;
  // sets active on each thickness row: zaptr[nt+1], zaset[]
  Region zaptr, zaset;
  // standard assembly: first overlapping function and overlap count per 1D
  // function, first function of every nonzero thickness span, the cells of each span
  Region a1f, a1c, a2f, a2c, zs_first, zs_cptr, zs_cell;
  // adjoint: ply of each accumulator slot per thickness row, slots finished after each row
  Region rowply, rowfin;
  // sets: material and (bucket) representative ply or (harmonic) harmonic index
  Region set_mat, set_aux, ply_mat, ply_set;
  // Kronecker scatter: tiles of whole in-plane rows (first in-plane nonzero
  // of each tile), chunks of thickness rows (first row of each chunk), the
  // sets each chunk keeps in LDS (chunk_sptr, chunk_set), and for every
  // active set of a row its LDS slot in the row's chunk (zaslot, parallel to
  // zaset); groups of consecutive chunks walked by one block (first chunk of
  // each), the distinct sets of each group (group_sptr, group_set) and each
  // chunk slot's index in its group's list (chunk_lset, parallel to chunk_set)
  Region tiles, chunk_ptr, chunk_sptr, chunk_set, zaslot, zchunk, group_ptr, group_sptr, group_set, chunk_lset;
  // curved shells, per in-plane element e = e1 + ne1*e2 and Gauss point
  // g = g1 + ng1*g2: gtab[e][g] = DF^{-T} (9, row-major) and the weight times
  // |det DF| (Gauss weights and half lengths included); rtab[e][g][b][3] =
  // (R, dR/dxi1, dR/dxi2) of local in-plane function b = b2*(p1+1) + b1
  Region gtab, rtab;
  // status words, zero after the upload, set (never cleared) by kernels that
  // find inputs the plan cannot honour; read and cleared by lam_check
  Region status;
  int64_t const_bytes = 0;  // end of the constant part
  // scratch: the fast assembly uses [const_bytes, fwd_end) (P only in LDS
  // mode, Eply only for harmonic plans evaluated per ply); the standard
  // assembly and the adjoint use the regions after it
  Region D, Ec, P, Qc, M, Eply, Qp, adj_part, adj_y, adj_cm;
  // material fields (fast scratch): bracket coefficients per set and in-plane
  // function, Ectl[s][is][81], and at every in-plane Gauss point, Epts[s][e][g][81]
  Region Ectl, Epts;
  int64_t fwd_end = 0;
  int64_t total = 0;
};

// Host plan construction (plan.cpp); lam_plan_create uses no tuning and
// min_nsc = 1.
lam_status plan_create(const lam_laminate_desc *d, const lam_tuning *tune, int min_nsc, lam_plan **out,
                       const lam_shell *shell = nullptr);
// Every field of a tuning within its documented range (NULL: automatic, valid).
bool tuning_ok(const lam_tuning *t);

// Kernel timing hooks (profile.cpp): a slot recorded around the dominant
// kernel of entry point `which` (0 assemble, 1 standard, 2 adjoint).
void *profile_begin(int which, void *stream);
void profile_end(void *slot, void *stream);

}  // namespace lam

struct lam_plan {
  // sizes
  int p1 = 0, p2 = 0, q = 0;
  int n1 = 0, n2 = 0, nt = 0, ns = 0;
  int ne1 = 0, ne2 = 0, nzc = 0;  // in-plane elements per direction, thickness cells
  int nzs = 0, max_span_cells = 0; // nonzero thickness knot spans, most cells in one span
  int adj_ok = 0;                   // every thickness pair touches at most two plies (adjoint supported)
  int ng1 = 0, ng2 = 0, ngz = 0;
  int n_ply = 0, n_mat = 0, n_sets = 0, set_mode = 0, n_harm = 0, maxact = 0;
  int64_t nnz1 = 0, nnz2 = 0, nnzz = 0, nnz = 0, nrows = 0;
  int n_tiles = 0, tile_k = 0;      // tiles of whole rows, at most tile_k in-plane nonzeros each
  int n_chunks = 0, chunk_sets = 0; // thickness-row chunks, at most chunk_sets sets in LDS each
  int n_groups = 0;                 // runs of consecutive chunks, one scatter block each
  int64_t kron_lds = 0;             // LDS bytes of the scatter kernel
  int kron_nsc = 0;                 // register mode: set slots per thread (0: LDS mode)
  int kron_threads = 256;           // scatter block size
  int harm_ply = 0;                 // harmonic sets evaluated per ply (scatter sets are the plies)
  int shell = 0;                    // curved extruded shell: per-point map gradients (gtab, rtab)
  int mat_field = 0;                // materials vary over the plane (C per in-plane function)
  int64_t kron_lds_q = 0, kron_lds_p = 0;  // LDS bytes of the Q and P parts (output buffer follows)
  double jit[9] = {0};  // DF^{-T}, row-major
  double detj = 0.0;    // |det DF|

  lam::Layout L;
  std::vector<uint8_t> image;  // host image of the constant part of the workspace
};
