// batch.hip -- many laminates of uneven size, degree and ply count,
// assembled wave by wave.
//
// Every laminate keeps its own plan (tables, tiles, chunks, sets).  Its
// constant tables sit in the batch workspace for the whole batch; its scratch
// (per-set rotated tensors and brackets, moments, folded 1D coefficients) sits
// in a wave arena reused by every wave; its CSR values go to the caller's wave
// buffer.  A wave is a run of laminates whose values and scratch fit the budget.
//
// A wave runs as these launches on one stream (all capturable in a HIP graph):
//   k_batch_prep   one block per small item: the rotated tensors and brackets
//                  of a laminate's sets (and the bucket check of its plies), or
//                  four of its folded 1D coefficients (one wave each);
//   k_batch_p2d    one block per 256 in-plane nonzeros of any laminate: the
//                  set-independent 2D moments (the scatter contracts P from them);
//   k_batch_kron_grid, once per scatter block size (64, 128, 192, 256 threads,
//                  the laminates' tile widths): one block per item (one tile of
//                  whole in-plane rows x one group of consecutive thickness
//                  chunks of one laminate).  A size's items are cut into eight
//                  contiguous ranges of equal output bytes, one per XCD; block b
//                  takes item b / 8 of range b mod 8 (blocks go to the XCDs in
//                  turn), so each XCD writes long contiguous runs of the CSR
//                  values and no cache line is written from two L2s.
// The device code of every item is the single-laminate path's (device.h):
// each laminate's values are bit for bit those of lam_assemble on its plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "device.h"

using lamdev::Dev;
using namespace lamdev;

struct lam_batch {
  int n = 0;
  std::vector<lam_plan *> plans;
  std::vector<int64_t> const_off;    // laminate tables in the batch workspace
  std::vector<int64_t> scratch_off;  // laminate scratch inside the wave arena
  std::vector<int64_t> c_off, t_off; // offsets (doubles) into the packed C and theta arrays
  std::vector<int> wave;             // wave of every laminate
  std::vector<int64_t> vals_off;     // offset (doubles) of its values in the wave buffer
  int n_waves = 0;
  std::vector<int> wave_first, wave_count;
  std::vector<int64_t> wave_vals;    // doubles of values per wave
  int64_t total_nnz = 0;
  // device layout of the batch workspace
  int64_t tables_bytes = 0, arena_off = 0, arena_bytes = 0;
  int64_t devs_off = 0, meta_off = 0, items_off = 0, status_off = 0, total = 0;
  // per wave: first item and count of the prep, 2D and scatter lists, and the
  // scatter list's eight per-XCD ranges (9 bounds, relative to its first item)
  std::vector<int64_t> wave_prep_off, wave_p2d_off, wave_kron_off;
  std::vector<int> wave_prep_n, wave_p2d_n, wave_kron_n;
  std::vector<int> wave_xcd;  // 9 per wave
  std::vector<int4> items;    // all lists of all waves, concatenated
  int64_t lds_bytes = 0;
};

namespace {

constexpr int BATCH_THREADS = 256;
constexpr int ITEM_ROTATE = 0, ITEM_Q1D = 1;
constexpr int N_XCD = 8;  // blocks are dispatched round-robin over the 8 XCDs
constexpr int N_GROUPS = 4;  // scatter block sizes 64, 128, 192, 256

int64_t a256(int64_t x) { return (x + 255) & ~int64_t(255); }

// Host view of a plan table (the image uploaded to the workspace).
template <class T>
const T *table(const lam_plan *p, const lam::Region &r) {
  return reinterpret_cast<const T *>(p->image.data() + r.off);
}

// Per-laminate metadata the kernel reads next to its Dev.
struct Meta {
  int64_t c_off, t_off, vals_off, pad;
};

struct BatchArgs {
  const Dev *__restrict__ devs;
  const Meta *__restrict__ meta;
  const int4 *__restrict__ items;  // this launch's list
  int n_items;
  int xcd_bound[N_XCD + 1];        // scatter: per-XCD item ranges
  const double *C_all, *th_all;
  double *vals;
};

// One block per prep item: {lam, ITEM_ROTATE, 0, 0} or {lam, ITEM_Q1D, i, 0}.
__global__ void __launch_bounds__(BATCH_THREADS) k_batch_prep(BatchArgs a) {
  const int4 w = a.items[blockIdx.x];
  const Dev &d = a.devs[w.x];
  const Meta m = a.meta[w.x];
  const double *th = a.th_all + m.t_off;
  if (w.y == ITEM_ROTATE) {
    for (int s = threadIdx.x; s < std::max(d.n_sets, d.n_ply); s += BATCH_THREADS) {
      check_ply(d, th, s);
      rotate_one(d, a.C_all + m.c_off, th, s);
    }
  } else {
    q1d_wave(d, th, (int64_t)w.z * (BATCH_THREADS / 64) + threadIdx.x / 64, threadIdx.x & 63);
  }
}

// One block per 2D item {lam, i, 0, 0}: in-plane nonzeros 256 i .. 256 i + 255.
__global__ void __launch_bounds__(BATCH_THREADS) k_batch_p2d(BatchArgs a) {
  const int4 w = a.items[blockIdx.x];
  const Dev &d = a.devs[w.x];
  p2d_one(d, d.Ec, d.P, d.M, (int64_t)w.y * BATCH_THREADS + threadIdx.x, 0);  // moments only
}

// The scatter: block b takes item b / 8 of XCD b % 8's range, the hardware
// dispatcher being the queue.
__global__ void __launch_bounds__(BATCH_THREADS) k_batch_kron_grid(BatchArgs a) {
  extern __shared__ double lds[];
  const int x = (int)(blockIdx.x % N_XCD), j = (int)(blockIdx.x / N_XCD);
  const int first = a.xcd_bound[x], count = a.xcd_bound[x + 1] - first;
  if (j >= count) return;
  const int4 wv = a.items[first + j];
  const Dev &d = a.devs[wv.x];
  kron_group<2, false>(d, d.Qc, a.vals + a.meta[wv.x].vals_off, wv.y, wv.z, lds, threadIdx.x, (int)blockDim.x);
}

// OR of every laminate's status words into *out (bit 0: a bucket set's plies
// disagree, bit 1: harmonic5 coupling, as lam_check), which are cleared.
__global__ void __launch_bounds__(BATCH_THREADS) k_batch_status(const Dev *__restrict__ devs, int n, int *out) {
  __shared__ int flags[BATCH_THREADS];
  int f = 0;
  for (int i = threadIdx.x; i < n; i += BATCH_THREADS) {
    int *st = devs[i].status;
    f |= (st[0] ? 1 : 0) | (st[1] ? 2 : 0);
    st[0] = 0;
    st[1] = 0;
  }
  flags[threadIdx.x] = f;
  __syncthreads();
  for (int h = BATCH_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) flags[threadIdx.x] |= flags[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = flags[0];
}

}  // namespace

extern "C" LAM_API void lam_batch_destroy(lam_batch *b) {
  if (!b) return;
  for (lam_plan *p : b->plans) lam_plan_destroy(p);
  delete b;
}

extern "C" LAM_API lam_status lam_batch_create(int32_t n, const lam_laminate_desc *descs, int64_t wave_bytes,
                                               lam_batch **out) {
  return lam_batch_create_tuned(n, descs, nullptr, wave_bytes, out);
}

extern "C" LAM_API lam_status lam_batch_create_tuned(int32_t n, const lam_laminate_desc *descs,
                                                     const lam_tuning *tunings, int64_t wave_bytes, lam_batch **out) {
  if (!out || !descs || n < 1) return LAM_EINVAL;
  *out = nullptr;
  lam_batch *B = new (std::nothrow) lam_batch();
  if (!B) return LAM_EINVAL;
  B->n = n;
  int64_t cbytes = 0, ctot = 0, ttot = 0;
  for (int i = 0; i < n; ++i) {
    lam_plan *p = nullptr;
    lam_tuning t = tunings ? tunings[i] : lam_tuning{0, 0, 0, 0};
    if (!lam::tuning_ok(&t)) {
      lam_batch_destroy(B);
      return LAM_EINVAL;
    }
    t.set_slots = 2;
    lam_status st = lam::plan_create(&descs[i], &t, 2, &p);
    if (st != LAM_OK) {
      lam_batch_destroy(B);
      return st;
    }
    B->plans.push_back(p);
    // the scatter kernel holds exactly two set slots per thread; harmonic
    // sets evaluated per ply (their per-ply tensors) are not batched
    if (p->kron_nsc != 2 || 3 * p->tile_k > BATCH_THREADS || p->harm_ply) {
      lam_batch_destroy(B);
      return LAM_EUNSUP;
    }
    B->const_off.push_back(cbytes);
    cbytes = a256(cbytes + p->L.const_bytes);
    B->c_off.push_back(ctot);
    B->t_off.push_back(ttot);
    ctot += 36 * (int64_t)p->n_mat;
    ttot += p->n_ply;
    B->total_nnz += p->nnz;
    B->lds_bytes = std::max<int64_t>(B->lds_bytes, p->kron_lds);
  }
  B->tables_bytes = cbytes;
  // waves: consecutive laminates whose values plus scratch fit wave_bytes
  B->wave.assign(n, 0);
  B->vals_off.assign(n, 0);
  B->scratch_off.assign(n, 0);
  int64_t vcur = 0, scur = 0, arena = 0;
  for (int i = 0; i < n; ++i) {
    const lam_plan *p = B->plans[i];
    const int64_t vb = 8 * p->nnz, sb = a256(p->L.fwd_end - p->L.const_bytes);
    if (B->n_waves == 0 || (wave_bytes > 0 && vcur > 0 && 8 * vcur + scur + vb + sb > wave_bytes)) {
      B->wave_first.push_back(i);
      B->wave_count.push_back(0);
      B->wave_vals.push_back(0);
      ++B->n_waves;
      vcur = scur = 0;
    }
    B->wave[i] = B->n_waves - 1;
    B->vals_off[i] = vcur;
    B->scratch_off[i] = scur;
    B->wave_vals.back() = vcur + p->nnz;
    vcur += (p->nnz + 31) & ~int64_t(31);  // 256-byte aligned starts
    scur += sb;
    B->wave_count.back() += 1;
    arena = std::max(arena, scur);
  }
  // work lists per wave: prep items, 2D items, scatter items (+ per-XCD ranges)
  for (int w = 0; w < B->n_waves; ++w) {
    const int f = B->wave_first[w], c = B->wave_count[w];
    B->wave_prep_off.push_back((int64_t)B->items.size());
    for (int i = f; i < f + c; ++i) {
      const lam_plan *p = B->plans[i];
      B->items.push_back(make_int4(i, ITEM_ROTATE, 0, 0));
      const int64_t nq = p->nnzz * std::max(p->kron_nsc, 1), per = BATCH_THREADS / 64;  // a wave per entry
      for (int64_t j = 0; j < (nq + per - 1) / per; ++j) B->items.push_back(make_int4(i, ITEM_Q1D, (int)j, 0));
    }
    B->wave_prep_n.push_back((int)((int64_t)B->items.size() - B->wave_prep_off.back()));
    B->wave_p2d_off.push_back((int64_t)B->items.size());
    for (int i = f; i < f + c; ++i) {
      const int np = (int)((B->plans[i]->nnz2 + BATCH_THREADS - 1) / BATCH_THREADS);
      for (int j = 0; j < np; ++j) B->items.push_back(make_int4(i, j, 0, 0));
    }
    B->wave_p2d_n.push_back((int)((int64_t)B->items.size() - B->wave_p2d_off.back()));
    // scatter items grouped by block size (the laminate's scatter threads),
    // each group cut into eight ranges of equal output bytes
    for (int T = 64; T <= BATCH_THREADS; T += 64) {
      B->wave_kron_off.push_back((int64_t)B->items.size());
      std::vector<double> cum(1, 0.0);  // output doubles before each item
      for (int i = f; i < f + c; ++i) {
        const lam_plan *p = B->plans[i];
        if (p->kron_threads != T) continue;
        const int *tiles = table<int>(p, p->L.tiles), *zrow = table<int>(p, p->L.zrow);
        const int *chunk = table<int>(p, p->L.chunk_ptr), *group = table<int>(p, p->L.group_ptr);
        for (int t = 0; t < p->n_tiles; ++t)
          for (int g = 0; g < p->n_groups; ++g) {
            B->items.push_back(make_int4(i, t, g, 0));
            cum.push_back(cum.back() + 9.0 * (tiles[t + 1] - tiles[t]) *
                                           (zrow[chunk[group[g + 1]]] - zrow[chunk[group[g]]]));
          }
      }
      const int nk = (int)cum.size() - 1;
      B->wave_kron_n.push_back(nk);
      int j = 0;
      for (int x = 0; x <= N_XCD; ++x) {
        const double target = cum.back() * x / N_XCD;
        while (j < nk && cum[j] < target) ++j;
        B->wave_xcd.push_back(x == N_XCD ? nk : j);
      }
    }
  }
  // batch workspace: tables | arena | Dev[n] | Meta[n] | items | status word
  int64_t off = a256(B->tables_bytes);
  B->arena_off = off;
  B->arena_bytes = a256(arena);
  off += B->arena_bytes;
  B->devs_off = off;
  off = a256(off + (int64_t)sizeof(Dev) * n);
  B->meta_off = off;
  off = a256(off + (int64_t)sizeof(Meta) * n);
  B->items_off = off;
  off = a256(off + (int64_t)sizeof(int4) * B->items.size());
  B->status_off = off;
  off = a256(off + (int64_t)sizeof(int));
  B->total = off;
  *out = B;
  return LAM_OK;
}

extern "C" LAM_API lam_status lam_batch_info(const lam_batch *b, int32_t *n_waves, int64_t *ws_bytes,
                                             int64_t *max_wave_vals, int64_t *total_nnz) {
  if (!b) return LAM_EINVAL;
  if (n_waves) *n_waves = b->n_waves;
  if (ws_bytes) *ws_bytes = b->total;
  if (max_wave_vals) *max_wave_vals = *std::max_element(b->wave_vals.begin(), b->wave_vals.end());
  if (total_nnz) *total_nnz = b->total_nnz;
  return LAM_OK;
}

extern "C" LAM_API lam_status lam_batch_laminate(const lam_batch *b, int32_t i, int32_t *wave, int64_t *vals_offset,
                                                 int64_t *nnz, int64_t *n_rows, int64_t *C_offset,
                                                 int64_t *theta_offset) {
  if (!b || i < 0 || i >= b->n) return LAM_EINVAL;
  const lam_plan *p = b->plans[i];
  if (wave) *wave = b->wave[i];
  if (vals_offset) *vals_offset = b->vals_off[i];
  if (nnz) *nnz = p->nnz;
  if (n_rows) *n_rows = p->nrows;
  if (C_offset) *C_offset = b->c_off[i];
  if (theta_offset) *theta_offset = b->t_off[i];
  return LAM_OK;
}

extern "C" LAM_API lam_status lam_batch_upload(const lam_batch *b, void *ws, int64_t ws_bytes, void *stream) {
  if (!b || !ws) return LAM_EINVAL;
  if (ws_bytes < b->total) return LAM_ESIZE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return LAM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(ws);
  std::vector<Dev> devs(b->n);
  std::vector<Meta> meta(b->n);
  for (int i = 0; i < b->n; ++i) {
    const lam_plan *p = b->plans[i];
    if (hipMemcpyAsync(base + b->const_off[i], p->image.data(), p->L.const_bytes, hipMemcpyHostToDevice, s) !=
        hipSuccess)
      return LAM_EHIP;
    devs[i] = lamdev::make_dev(p, base + b->const_off[i], base + b->arena_off + b->scratch_off[i]);
    meta[i].c_off = b->c_off[i];
    meta[i].t_off = b->t_off[i];
    meta[i].vals_off = b->vals_off[i];
    meta[i].pad = 0;
  }
  // host arrays must outlive the asynchronous copies: copy synchronously
  if (hipMemcpyAsync(base + b->devs_off, devs.data(), sizeof(Dev) * devs.size(), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(base + b->meta_off, meta.data(), sizeof(Meta) * meta.size(), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(base + b->items_off, b->items.data(), sizeof(int4) * b->items.size(), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return LAM_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? LAM_OK : LAM_EHIP;
}

extern "C" LAM_API lam_status lam_batch_pattern(const lam_batch *b, const void *ws, int64_t ws_bytes, int32_t i,
                                                int64_t *rowptr, int32_t *colind, void *stream) {
  if (!b || !ws || i < 0 || i >= b->n) return LAM_EINVAL;
  if (ws_bytes < b->total) return LAM_ESIZE;
  const lam_plan *p = b->plans[i];
  // the pattern kernels read constant tables only
  return lam_pattern(p, static_cast<const char *>(ws) + b->const_off[i], p->L.total, rowptr, colind, stream);
}

extern "C" LAM_API lam_status lam_batch_assemble(const lam_batch *b, void *ws, int64_t ws_bytes, int32_t wave,
                                                 const double *C_all, const double *theta_all, double *vals_wave,
                                                 int64_t vals_len, void *stream) {
  if (!b || !ws || !C_all || !theta_all || !vals_wave) return LAM_EINVAL;
  if (wave < 0 || wave >= b->n_waves) return LAM_EINVAL;
  if (ws_bytes < b->total || vals_len < b->wave_vals[wave]) return LAM_ESIZE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(ws);
  const int4 *items = reinterpret_cast<const int4 *>(base + b->items_off);
  BatchArgs a;
  a.devs = reinterpret_cast<const Dev *>(base + b->devs_off);
  a.meta = reinterpret_cast<const Meta *>(base + b->meta_off);
  a.C_all = C_all;
  a.th_all = theta_all;
  a.vals = vals_wave;
  void *prof = lam::profile_begin(3, stream);
  a.items = items + b->wave_prep_off[wave];
  a.n_items = b->wave_prep_n[wave];
  hipLaunchKernelGGL(k_batch_prep, dim3(a.n_items), dim3(BATCH_THREADS), 0, s, a);
  a.items = items + b->wave_p2d_off[wave];
  a.n_items = b->wave_p2d_n[wave];
  hipLaunchKernelGGL(k_batch_p2d, dim3(a.n_items), dim3(BATCH_THREADS), 0, s, a);
  for (int g = 0; g < N_GROUPS; ++g) {
    const int gi = N_GROUPS * wave + g;
    if (b->wave_kron_n[gi] == 0) continue;
    a.items = items + b->wave_kron_off[gi];
    a.n_items = b->wave_kron_n[gi];
    for (int x = 0; x <= N_XCD; ++x) a.xcd_bound[x] = b->wave_xcd[(N_XCD + 1) * gi + x];
    const dim3 block(64 * (g + 1));
    int most = 0;
    for (int x = 0; x < N_XCD; ++x) most = std::max(most, a.xcd_bound[x + 1] - a.xcd_bound[x]);
    hipLaunchKernelGGL(k_batch_kron_grid, dim3(N_XCD * most), block, (size_t)b->lds_bytes, s, a);
  }
  lam::profile_end(prof, stream);
  return hipGetLastError() == hipSuccess ? LAM_OK : LAM_EHIP;
}

extern "C" LAM_API lam_status lam_batch_check(const lam_batch *b, void *ws, int64_t ws_bytes, int32_t *flags,
                                              void *stream) {
  if (!b || !ws || !flags) return LAM_EINVAL;
  if (ws_bytes < b->total) return LAM_ESIZE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(ws);
  int *out = reinterpret_cast<int *>(base + b->status_off);
  hipLaunchKernelGGL(k_batch_status, dim3(1), dim3(BATCH_THREADS), 0, s, reinterpret_cast<const Dev *>(base + b->devs_off),
                     b->n, out);
  int host = 0;
  if (hipMemcpyAsync(&host, out, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LAM_EHIP;
  *flags = host;
  return LAM_OK;
}
