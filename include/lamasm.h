/*
 * lamasm.h -- C ABI of the fast layered-stiffness assembly library (liblamasm.so).
 *
 * The library assembles the 3D Galerkin stiffness matrix K of a laminated
 * solid (Antolin, arXiv 1905.05417) on one gfx950 GPU:
 *
 *   K^{ij} = sum_l sum_{a,b in {1,2}} P_{l,ab}^{is js} Q_{l,ab}^{it jt}        (Sec. 3, eq. Km_2)
 *
 * P are 2D in-plane integrals (eq. P), computed once per set of plies sharing
 * a material and an orientation (or once per material and angular harmonic,
 * Remark 3), and Q are 1D through-thickness integrals per ply (eq. Q).  The
 * result is written into a preallocated CSR pattern.  A standard 3D
 * element-by-element assembly (Sec. 2.4) writes the same CSR for comparison,
 * and an adjoint maps dL/dK to dL/dC (materials) and dL/dtheta (plies).
 *
 * Conventions
 *  - Basis (Assumption 1): B^i = S^{is}(xi1,xi2) T^{it}(xi3), in-plane
 *    is = i1 + n1*i2 (tensor-product B-splines of degrees p1, p2), thickness
 *    functions it (B-splines of degree q).  Global function i = it*ns + is,
 *    degree of freedom 3*i + r (r = displacement component x,y,z), eq. a_0.
 *  - Geometry (Assumption 2, eq. extrusion): x = DF xi with a constant 3x3 map
 *    gradient DF (an affine extrusion; a box plate is diag(Lx, Ly, H)), or a
 *    curved mid-surface extruded along a vector (lam_plan_create_shell).
 *  - Plies (Sec. 2.3): ply l occupies xi3 in [iface[l], iface[l+1]],
 *    iface[0] = 0 < ... < iface[n_ply] = 1, ply 0 at the bottom.
 *  - Materials: 6x6 matrices in material axes, Voigt order
 *    (11,22,33,12,13,23) with engineering shears (eq. D), row-major, used as
 *    given (no symmetrisation).  Ply l uses material ply_mat[l] rotated by
 *    theta[l] radians counterclockwise about +e3 (fibre axis (cos, sin, 0)).
 *  - CSR: int64 row pointers, int32 column indices, FP64 values; columns of a
 *    row ascending; the pattern is structural (all pairs of functions whose
 *    supports share a cell, times dense 3x3 blocks) and keeps explicit zeros.
 *
 * Ownership and streams
 *  - The caller owns every device buffer: the workspace, C, theta, vals,
 *    rowptr, colind, gradients.  A plan owns host memory only.
 *  - Device entry points are asynchronous on the given stream (a hipStream_t
 *    passed as void*; NULL is the default stream), never allocate device
 *    memory and never synchronise.  Errors of earlier asynchronous work may
 *    surface as LAM_EHIP on a later call.
 *  - One workspace per stream that uses it concurrently.
 */
#ifndef LAMASM_H
#define LAMASM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define LAM_API __attribute__((visibility("default")))
#else
#define LAM_API
#endif

typedef int32_t lam_status;
#define LAM_OK 0
#define LAM_EINVAL (-1)  /* null pointer, bad enum, bad count */
#define LAM_EKNOT (-2)   /* knot vector not open on [0,1], decreasing, or degree out of range */
#define LAM_EPLY (-3)    /* interfaces not strictly increasing from 0 to 1, bad ply/material index */
#define LAM_EMAT (-4)    /* non-finite material or angle, singular map gradient */
#define LAM_ESIZE (-5)   /* workspace or output length does not match the plan */
#define LAM_EHIP (-6)    /* HIP runtime error (launch or an earlier asynchronous fault) */
#define LAM_EUNSUP (-7)  /* supported by the method but not by this build (limits below) */
#define LAM_ESCRATCH (-8) /* the plan needs more scratch than lam_assemble_static's static buffer */

/* How plies are grouped into the sets that share one 2D operator P.
 *  BUCKET:     one set per distinct (material, angle) pair, the grouping read
 *              from desc.ply_theta at plan time (Sec. 3, reuse per distinct
 *              orientation).  The angles passed at assembly must agree within
 *              each set; the set's angle is that of its first ply (a
 *              disagreement raises LAM_CHECK_BUCKET_ANGLES, see lam_check).
 *  HARMONIC5:  one set per (material, harmonic), harmonics {1, cos 2t,
 *              sin 2t, cos 4t, sin 4t}: exact for any angles when each
 *              material has no coupling between {11,22,33,12} and {13,23}
 *              (orthotropic or monoclinic about the ply plane), Remark 3;
 *              a coupled material raises LAM_CHECK_HARMONIC5_COUPLING.
 *  HARMONIC9:  harmonics up to order 4 including odd ones: exact for any 6x6.
 *  PLY:        one set per ply: exact for any angles passed at assembly
 *              (no plan-time angles needed).  The scatter forms each set's 2D
 *              operator from set-independent moments, so many sets cost little.
 */
#define LAM_SETS_BUCKET 0
#define LAM_SETS_HARMONIC5 1
#define LAM_SETS_HARMONIC9 2
#define LAM_SETS_PLY 3

/* Limits of this build: 1 <= p1, p2 <= 4, 1 <= q <= 4, Gauss points per
 * direction 1..8, n_ply <= 4096, n_mat <= 64, nnz < 2^62, columns < 2^31. */

typedef struct {
  int32_t p1, nk1;          /* in-plane degree and open knot vector (nk1 knots) along xi1 */
  const double *k1;
  int32_t p2, nk2;          /* same along xi2 */
  const double *k2;
  int32_t q, nk3;           /* thickness degree and knot vector along xi3 */
  const double *k3;
  double jac[9];            /* DF, row-major: jac[3*a+b] = d x_a / d xi_b */
  int32_t n_ply;
  const double *iface;      /* n_ply+1 interfaces */
  const int32_t *ply_mat;   /* n_ply material indices in [0, n_mat) */
  int32_t n_mat;
  const double *ply_theta;  /* n_ply angles (radians), host; required for BUCKET, ignored otherwise */
  int32_t ng1, ng2, ngz;    /* Gauss points per in-plane element direction and per thickness
                               cell (ply x thickness knot span); 0 selects degree+1 */
  int32_t set_mode;         /* LAM_SETS_* */
} lam_laminate_desc;

typedef struct lam_plan lam_plan;

/* Validates the descriptor and builds the host tables (knot spans, basis
 * values at Gauss points, in-plane / thickness / Kronecker patterns, set
 * grouping).  Host only; copies everything it needs from desc. */
LAM_API lam_status lam_plan_create(const lam_laminate_desc *desc, lam_plan **out);
LAM_API void lam_plan_destroy(lam_plan *plan);

/* Scatter tuning (performance only: the values of K do not depend on it).
 * Zero fields select the automatic choice. */
typedef struct {
  int32_t tile_k;         /* in-plane nonzeros per scatter tile, <= 85 (tiles hold whole rows, so
                             it is widened to the longest row); automatic: about 85 */
  int32_t set_slots;      /* register-mode set slots per chunk of thickness rows: 1, 2, 4 or 8;
                             automatic: 2 (raised to the most sets active on one row) */
  int32_t target_blocks;  /* thickness rows are chunked so the scatter has about this many
                             blocks; automatic: 6144 */
  int32_t lds_kib;        /* LDS budget of the LDS-mode scatter, <= 160; automatic: 80 */
} lam_tuning;

/* lam_plan_create with explicit scatter tuning (tuning may be NULL). */
LAM_API lam_status lam_plan_create_tuned(const lam_laminate_desc *desc, const lam_tuning *tuning, lam_plan **out);

/* Curved laminated shells (Sec. 2.3, Assumption 2, eq. extrusion;
 * Assumption 3): the laminate's in-plane map is the extrusion of a
 * mid-surface, F(xi) = S(xi1, xi2) + xi3 a, with S = sum_i R^i(xi1, xi2) ctrl_i
 * over the in-plane basis of the descriptor (its knots and degrees).  Without
 * weights R^i are the B-splines; with weights they are NURBS,
 * R^i = w_i N^i / sum_k w_k N^k (Sec. 2.2), for the geometry and the
 * displacement alike.  The map gradient DF = [dS/dxi1 | dS/dxi2 | a] varies
 * over the plane but not through the thickness, which is what the split of
 * Sec. 3 needs; desc.jac is not used.  Plies may also carry materials that
 * vary over the plane: with mat_field set, C holds one 6x6 per material and
 * in-plane function (n_mat * n1 * n2 matrices, material-major), and ply l uses
 * C_{mat(l)}(xi) = sum_i R^i(xi) C_{mat(l), i} rotated by theta_l.
 * Limits: material fields take BUCKET or PLY sets (LAM_EUNSUP otherwise), no
 * adjoint or standard assembly (LAM_EUNSUP); their matrix-free product and CG
 * read the P of each set integrated with the field inside; curved shells with
 * constant materials support every entry point except the batch.
 * lam_plan_create_shell returns LAM_EMAT for a non-finite control point,
 * weight or extrusion vector, a weight <= 0 or a map gradient that is
 * singular at an in-plane Gauss point. */
typedef struct {
  const double *ctrl;     /* n1*n2 control points (x, y, z), in-plane function order i1 + n1*i2 (host) */
  const double *weights;  /* NULL (B-splines) or n1*n2 positive weights (NURBS) (host) */
  double a[3];            /* extrusion vector */
  int32_t mat_field;      /* 0: C holds n_mat 6x6; 1: n_mat*n1*n2 of them (one per in-plane function) */
} lam_shell;

LAM_API lam_status lam_plan_create_shell(const lam_laminate_desc *desc, const lam_shell *shell,
                                         const lam_tuning *tuning, lam_plan **out);

/* Sizes: rows of K (3*n), nonzeros, workspace bytes, number of sets, and the
 * number of plies and materials the device arrays must hold.  Any pointer may be NULL. */
LAM_API lam_status lam_plan_info(const lam_plan *plan, int64_t *n_rows, int64_t *nnz, int64_t *ws_bytes,
                                 int32_t *n_sets, int32_t *n_ply, int32_t *n_mat);

/* Copies the plan's constant tables into the device workspace `ws`
 * (ws_bytes from lam_plan_info, 256-byte aligned).  Must precede every other
 * device call on that workspace; asynchronous on `stream`. */
LAM_API lam_status lam_plan_upload(const lam_plan *plan, void *ws, int64_t ws_bytes, void *stream);

/* Reads and clears the workspace's status flags (synchronizes the stream;
 * not for HIP graph capture).  The fast assembly checks its inputs against
 * the plan on the device, since C and theta live there, and raises a flag
 * instead of failing; a flag stays set until this call.  *flags (host)
 * receives the OR of:
 *  LAM_CHECK_BUCKET_ANGLES: a BUCKET plan was given a theta in which the
 *    plies of one set differ; every ply of the set was rotated by the angle
 *    of the set's first ply, so the values are not K(theta) (Sec. 3: one 2D
 *    operator per distinct orientation).  Use LAM_SETS_PLY or a harmonic
 *    mode for angles that change per ply.
 *  LAM_CHECK_HARMONIC5_COUPLING: a HARMONIC5 plan was given a material with
 *    an entry coupling {11,22,33,12} with {13,23} above 1e-13 of its largest
 *    entry; its rotation has odd harmonics that the five terms of the Remark
 *    on orientations omit.  Use LAM_SETS_HARMONIC9.
 * Returns LAM_OK (whatever the flags) or a size / HIP error. */
#define LAM_CHECK_BUCKET_ANGLES 1
#define LAM_CHECK_HARMONIC5_COUPLING 2
LAM_API lam_status lam_check(const lam_plan *plan, void *ws, int64_t ws_bytes, int32_t *flags, void *stream);

/* Writes the CSR pattern: rowptr[n_rows+1] (int64) and colind[nnz] (int32). */
LAM_API lam_status lam_pattern(const lam_plan *plan, const void *ws, int64_t ws_bytes, int64_t *rowptr,
                               int32_t *colind, void *stream);

/* Fast 2D x 1D assembly (Sec. 3): vals[nnz] in the order of lam_pattern.
 * C: device, n_mat*36 doubles; theta: device, n_ply doubles (radians).
 * Every value of vals is overwritten. */
LAM_API lam_status lam_assemble(const lam_plan *plan, void *ws, int64_t ws_bytes, const double *C,
                                const double *theta, double *vals, int64_t nnz, void *stream);

/* lam_assemble for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same values, bit for bit, but the assembly's
 * scratch (set tensors, bracket coefficients, in-plane moments, thickness
 * coefficients: bytes [const part, fast-scratch end) of the workspace layout)
 * lives in a static device array of LAM_STATIC_SCRATCH_MIB MiB that the
 * library holds on every GPU it runs on until the process ends.  ws needs only
 * the plan's constant tables: any ws_bytes from the constant part's size up
 * (lam_plan_info's ws_bytes always suffices; lam_plan_upload fills it) and
 * nothing in it is written except the status words of lam_check.  Calls that
 * allocate nothing: no hipMalloc, no hipFree, no allocating library routine.
 * Every call on one GPU shares that GPU's static array, so calls that overlap
 * on one GPU (concurrent streams, threads) race and must be serialized by the
 * caller.  LAM_ESCRATCH if the plan's scratch exceeds the array (about
 * 288 B per in-plane nonzero: up to ~460,000 in-plane nonzeros, e.g. degree 2
 * on 128x128 elements), LAM_EHIP if the array's address cannot be obtained. */
#define LAM_STATIC_SCRATCH_MIB 128
LAM_API lam_status lam_assemble_static(const lam_plan *plan, void *ws, int64_t ws_bytes, const double *C,
                                       const double *theta, double *vals, int64_t nnz, void *stream);

/* Standard 3D assembly (Sec. 2.4): element by element over every
 * (in-plane element x ply x thickness knot span) cell with the tensor Gauss
 * rule, element matrices added into the same CSR (colour by colour, no
 * atomics: the values do not depend on the schedule).  Same arguments and
 * output as lam_assemble; LAM_EUNSUP for in-plane material fields. */
LAM_API lam_status lam_assemble_standard(const lam_plan *plan, void *ws, int64_t ws_bytes, const double *C,
                                         const double *theta, double *vals, int64_t nnz, void *stream);

/* Adjoint of lam_assemble: given G = dL/dvals (device, nnz doubles in the
 * order of lam_pattern), writes grad_C = dL/dC (device, n_mat*36, each of the
 * 36 entries treated as independent) and grad_theta = dL/dtheta (device,
 * n_ply, per radian).  K is linear in each ply's rotated tensor D_l (eq. Km_0),
 * so dL/dD_l is a contraction of G with the thickness operators Q_l and the
 * in-plane moments of the basis; dK is never formed. */
LAM_API lam_status lam_adjoint(const lam_plan *plan, void *ws, int64_t ws_bytes, const double *C,
                               const double *theta, const double *grad_vals, int64_t nnz, double *grad_C,
                               double *grad_theta, void *stream);

/* Matrix-free product y = K u (eq. Km_2 applied to a vector): the Kronecker
 * split of lam_assemble evaluated against u without forming K.  u and y:
 * device, n_rows doubles in the row order of lam_pattern; y is overwritten.
 * fixed: NULL, or device bytes per row (nonzero = Dirichlet row) for the
 * eliminated operator y = P K P u + (I - P) u, P the projection on the free
 * rows.  Register-mode plans with one or two set slots (every bucket and
 * per-ply plan with the automatic slot count); with an in-plane material
 * field each call first integrates every set's P with the field inside (as
 * lam_assemble does) and the product reads it.  LAM_EUNSUP otherwise,
 * LAM_ESIZE if n_rows is not the plan's row count.  The rounding order
 * differs from multiplying the assembled K. */
LAM_API lam_status lam_apply(const lam_plan *plan, void *ws, int64_t ws_bytes, const double *C, const double *theta,
                             const double *u, const uint8_t *fixed, int64_t n_rows, double *y, void *stream);

/* Conjugate gradients for K x = b with homogeneous Dirichlet rows eliminated:
 * solves (P K P + I - P) x = P b (fixed as for lam_apply, NULL for none, then
 * K itself must be nonsingular on the data), starting from the x given
 * (device, n_rows doubles, overwritten), until ||r|| <= tol ||P b|| or
 * max_iter iterations, preconditioned by thickness lines: for every in-plane
 * function, the operator's block coupling all its thickness functions and
 * displacement components (banded, half bandwidth 3q + 2), taken from the
 * split of Sec. 3 at the in-plane diagonal (the 1D integrals times the
 * diagonal's 2D ones) and factored once by a banded Cholesky.  Every
 * product is lam_apply's; vector updates and dot products are kernels of
 * their own with device-side scalars.  work: device, at least
 * lam_cg_work_bytes(plan) bytes, 8-byte aligned.  Unlike the other
 * entry points it waits on the stream, after every 8 iterations (to test the
 * residual), so up to 7 iterations may run past the tolerance; *iters and
 * *rel_res (host) receive the iteration count and the final relative
 * residual.  LAM_ESIZE for a short work buffer or a wrong
 * n_rows; LAM_EUNSUP as for lam_apply. */
LAM_API int64_t lam_cg_work_bytes(const lam_plan *plan);
LAM_API lam_status lam_cg(const lam_plan *plan, void *ws, int64_t ws_bytes, const double *C, const double *theta,
                          const uint8_t *fixed, const double *b, double *x, int64_t n_rows, void *work,
                          int64_t work_bytes, double tol, int32_t max_iter, int32_t *iters, double *rel_res,
                          void *stream);

/* Rank-one adjoint: the gradient of L = u^T K u (strain energy times two,
 * compliance) with respect to C and theta, i.e. lam_adjoint with
 * G = u u^T on the pattern of K, but G is never formed or read: each thread
 * forms its entries of G from u as it streams.  u: device, n_rows doubles in
 * the row order of lam_pattern (3 (i_t n_s + i_s) + component); grad_C and
 * grad_theta as for lam_adjoint.  LAM_ESIZE if n_rows is not the plan's row
 * count; LAM_EUNSUP where lam_adjoint is unsupported. */
LAM_API lam_status lam_adjoint_rank1(const lam_plan *plan, void *ws, int64_t ws_bytes, const double *C,
                                     const double *theta, const double *u, int64_t n_rows, double *grad_C,
                                     double *grad_theta, void *stream);

/* Batched assembly: many laminates (different meshes, degrees, ply counts,
 * materials) assembled wave by wave, each laminate's values exactly those of
 * lam_assemble on its own plan (Sec. 3 applied per laminate; the device code
 * is the same).
 *
 * lam_batch_create plans every descriptor (host only) and splits the
 * laminates, in the given order, into waves: runs of consecutive laminates
 * whose CSR values plus scratch fit wave_bytes (<= 0: one wave).  A laminate
 * larger than wave_bytes forms a wave of its own.  Fails with the first
 * failing descriptor's status, or LAM_EUNSUP for a laminate whose scatter
 * needs more than two set slots per thickness chunk (many distinct sets on
 * one row, e.g. harmonic sets: use lam_assemble for it).  Affine laminates
 * only (no curved shells).
 *
 * Device memory: one workspace of ws_bytes (lam_batch_info), 256-byte
 * aligned, holding every plan's constant tables, one scratch arena reused by
 * all waves, the work lists and a status word.  C_all packs the laminates'
 * n_mat*36 tensors and theta_all their n_ply angles at the offsets
 * lam_batch_laminate reports (device doubles).  Values of wave w go to
 * vals_wave (device, vals_len >= that wave's length <= max_wave_vals doubles),
 * laminate i at vals_offset (a multiple of 32 doubles) within its wave; gaps
 * between laminates are not written. */
typedef struct lam_batch lam_batch;

LAM_API lam_status lam_batch_create(int32_t n, const lam_laminate_desc *descs, int64_t wave_bytes, lam_batch **out);
/* The same with per-laminate scatter tuning (tunings: n entries, or NULL);
 * set_slots is fixed at 2 by the batched scatter. */
LAM_API lam_status lam_batch_create_tuned(int32_t n, const lam_laminate_desc *descs, const lam_tuning *tunings,
                                          int64_t wave_bytes, lam_batch **out);
LAM_API void lam_batch_destroy(lam_batch *batch);
LAM_API lam_status lam_batch_info(const lam_batch *batch, int32_t *n_waves, int64_t *ws_bytes,
                                  int64_t *max_wave_vals, int64_t *total_nnz);
/* Per laminate i: its wave, the offset of its values in that wave's buffer,
 * its nonzeros and rows, and its offsets into C_all and theta_all (doubles). */
LAM_API lam_status lam_batch_laminate(const lam_batch *batch, int32_t i, int32_t *wave, int64_t *vals_offset,
                                      int64_t *nnz, int64_t *n_rows, int64_t *C_offset, int64_t *theta_offset);
/* Copies every plan's tables, the per-laminate device views and descriptors and the
 * per-wave work lists (one item per block of each of a wave's launches: set and 1D
 * prep, 2D moments, scatter) to ws; synchronizes stream. */
LAM_API lam_status lam_batch_upload(const lam_batch *batch, void *ws, int64_t ws_bytes, void *stream);
/* CSR pattern of laminate i, as lam_pattern. */
LAM_API lam_status lam_batch_pattern(const lam_batch *batch, const void *ws, int64_t ws_bytes, int32_t i,
                                     int64_t *rowptr, int32_t *colind, void *stream);
/* Assembles every laminate of wave `wave`: a launch for the rotated tensors
 * and brackets of every laminate's sets and their folded 1D coefficients, a
 * launch for the 2D moments of all the wave's laminates, then one scatter
 * launch per scatter block size (at most four), each block one (tile, group
 * of thickness chunks) item, items cut into eight ranges of equal output
 * bytes, one per XCD.  Asynchronous; may be captured in a HIP graph (no
 * memset, no allocation, no host synchronization).  Waves share the scratch
 * arena: waves on different streams must not overlap. */
LAM_API lam_status lam_batch_assemble(const lam_batch *batch, void *ws, int64_t ws_bytes, int32_t wave,
                                      const double *C_all, const double *theta_all, double *vals_wave,
                                      int64_t vals_len, void *stream);
/* Reads and clears the status flags of every laminate (synchronizes stream):
 * *flags (host) receives the OR over the laminates of the LAM_CHECK_* bits of
 * lam_check, raised by any assembly since the last check (bucket sets whose
 * plies were given different angles in theta_all). */
LAM_API lam_status lam_batch_check(const lam_batch *batch, void *ws, int64_t ws_bytes, int32_t *flags,
                                   void *stream);

/* Kernel timing for measurement.  While enabled, every device entry point
 * records a pair of HIP events on its stream around its dominant kernel
 * (the Kronecker scatter of lam_assemble, the element kernels of
 * lam_assemble_standard, the streaming contraction of lam_adjoint and
 * lam_adjoint_rank1, the scatter of lam_batch_assemble, the product kernel
 * of lam_apply), and lam_assemble_standard also around the zero fill of its
 * output (a plain grid-stride store stream: the write rate the output's
 * allocation allows); no work is added or skipped.
 * lam_profile_read waits for the recorded events and returns the summed
 * milliseconds and the number of timed launches per slot (index 0 assemble,
 * 1 standard, 2 adjoint, 3 batch, 4 apply, 5 the standard's zero fill), then
 * clears them.  Up to 4096 launches are kept; later ones are not timed. */
#define LAM_PROFILE_SLOTS 6
LAM_API lam_status lam_profile_enable(int32_t on);
LAM_API lam_status lam_profile_read(double ms[LAM_PROFILE_SLOTS], int64_t launches[LAM_PROFILE_SLOTS]);

LAM_API const char *lam_status_string(lam_status s);

/* Library version, for diagnostics. */
LAM_API const char *lam_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LAMASM_H */
