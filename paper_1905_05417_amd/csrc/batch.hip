// batch.hip -- many laminates of uneven size, degree and ply count assembled
// by one persistent kernel per memory wave.
//
// Every laminate keeps its own plan (tables, tiles, chunks, sets).  Its
// constant tables sit in the batch workspace for the whole batch; its scratch
// (per-set rotated tensors, P, Q coefficients, moments) sits in a wave arena
// reused by every wave; its CSR values go to the caller's wave buffer.  A
// wave is a run of laminates whose values and scratch fit the budget.
//
// A wave runs as three launches on one stream (all capturable in a HIP graph):
//   k_batch_reset  clears the queue head, error flag and completion counters;
//   k_batch_prep   one block per small item: rotated tensors / harmonics of a
//                  laminate's sets, and 256 of its folded 1D coefficients;
//   k_batch        the persistent kernel, over a queue of
//                    p2d(b, i)  - 256 in-plane nonzeros of laminate b's 2D operators
//                    kron(b, L) - one scatter tile x chunk of b (needs every p2d(b, .))
//                  ordered p2d(b0), p2d(b1), kron(b0), p2d(b2), kron(b1), ...
//                  so the 2D work (arithmetic bound) of the next laminate
//                  overlaps the scatter (store bound) of the previous one.
// Blocks of the persistent kernel take items from an atomic head counter; a
// scatter item whose laminate's 2D items are not all finished waits on that
// laminate's completion counter.  Those items are earlier in the queue, so
// they were taken by running blocks, which wait on nothing; every wait ends.
// The wait is also bounded in time: past the bound the batch error flag is set,
// the item skipped, and every later wait of the launch returns at once.  Completion is released and acquired at agent
// scope (the per-XCD L2s are written back / invalidated by those fences).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "device.h"

using lamdev::Dev;

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
  int64_t devs_off = 0, meta_off = 0, items_off = 0, counters_off = 0, total = 0;
  std::vector<int64_t> wave_prep_off, wave_items_off;  // first prep / queue item of each wave
  std::vector<int> wave_prep_n, wave_items_n;
  std::vector<int4> items;               // all waves, concatenated
  int64_t lds_bytes = 0;
  int grid = 2048;  // persistent blocks
  mutable long long wall_khz = 100000;  // device constant-clock rate, read at upload
};

namespace {

constexpr int BATCH_THREADS = 256;
constexpr int LAM_BATCH_WAIT_MS = 500;  // a dependency wait longer than this is an error
constexpr int ITEM_ROTATE = 0, ITEM_Q1D = 1, ITEM_P2D = 2, ITEM_KRON = 3;

int64_t a256(int64_t x) { return (x + 255) & ~int64_t(255); }

// Per-laminate metadata the kernel reads next to its Dev.
struct Meta {
  int64_t c_off, t_off, vals_off;
  int n_p_items;
  int pad;
};

struct BatchArgs {
  const Dev *__restrict__ devs;
  const Meta *__restrict__ meta;
  const int4 *__restrict__ items;
  int n_items;
  int *counters;  // [0] queue head, [1] error flag, then per laminate: 2D items done
  const double *C_all, *th_all;
  double *vals;
  long long wait_ticks;  // longest wait of one item, in wall-clock ticks
};

__device__ inline int *lam_counter(const BatchArgs &a, int lam) { return a.counters + 2 + lam; }

// Thread 0: wait until *c >= target.  Polls with relaxed loads (no cache
// invalidation per poll: the caller's block issues one acquire fence after
// the wait) and gives up, setting the sticky error flag, after `ticks` of the
// constant-rate clock or as soon as any other wait of the launch has given up.
__device__ inline int wait_at_least(int *c, int target, int *err, long long ticks) {
  const long long t0 = wall_clock64();
  while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return 0;
    if (wall_clock64() - t0 > ticks) {
      atomicOr(err, 1);
      return 0;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return 1;
}

__global__ void k_batch_reset(int *counters, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) counters[i] = 0;
}

// One block per prep item: {lam, ITEM_ROTATE, 0, 0} or {lam, ITEM_Q1D, i, 0}.
__global__ void __launch_bounds__(BATCH_THREADS) k_batch_prep(BatchArgs a, const int4 *__restrict__ items) {
  const int4 w = items[blockIdx.x];
  const Dev &d = a.devs[w.x];
  const Meta m = a.meta[w.x];
  const double *th = a.th_all + m.t_off;
  if (w.y == ITEM_ROTATE) {
    for (int s = threadIdx.x; s < d.n_sets; s += BATCH_THREADS) lamdev::item_rotate_set(d, a.C_all + m.c_off, th, s);
  } else {
    const int64_t idx = (int64_t)w.z * BATCH_THREADS + threadIdx.x;
    if (idx < d.nnzz * lamdev::q1d_width(d)) lamdev::item_q1d(d, th, idx);
  }
}

// Control flow around every barrier is uniform and visibly so to the
// compiler: the item index, its fields and the wait result are broadcast
// through LDS and read into scalar registers (readfirstlane), and each
// iteration starts with a barrier, so the single-thread regions (the queue
// and counter atomics) never sit next to each other across the loop's
// back-edge.  Otherwise the structurizer may turn the loop into nested
// exec-masked loops in which the other lanes of thread 0's wave re-enter the
// loop-top barrier without thread 0.
__global__ void __launch_bounds__(BATCH_THREADS) k_batch(BatchArgs a) {
  extern __shared__ double lds[];
  __shared__ int s_item, s_ok;
  const int tid = threadIdx.x;
  for (;;) {
    __syncthreads();  // the previous item is finished by every thread (LDS reuse)
    if (tid == 0) s_item = atomicAdd(a.counters, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= a.n_items) break;
    const int4 wv = a.items[it];
    const int lam = __builtin_amdgcn_readfirstlane(wv.x), type = __builtin_amdgcn_readfirstlane(wv.y);
    const int wz = __builtin_amdgcn_readfirstlane(wv.z), ww = __builtin_amdgcn_readfirstlane(wv.w);
    const Dev &d = a.devs[lam];
    if (type == ITEM_P2D) {
      const int64_t k = (int64_t)wz * BATCH_THREADS + tid;
      if (k < d.nnz2) lamdev::item_p2d(d, d.Ec, d.P, d.M, k, 1);
      // completion: this thread's P writes visible device-wide, then count the item
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (tid == 0) __hip_atomic_fetch_add(lam_counter(a, lam), 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (tid == 0) s_ok = wait_at_least(lam_counter(a, lam), a.meta[lam].n_p_items, a.counters + 1, a.wait_ticks);
      __syncthreads();
      const int ok = __builtin_amdgcn_readfirstlane(s_ok);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (ok) {
        double *vals = a.vals + a.meta[lam].vals_off;
        if (d.kron_nsc == 1)
          lamdev::item_kron_reg<1>(d, d.Qc, vals, wz, ww, lds, tid, BATCH_THREADS);
        else
          lamdev::item_kron_reg<2>(d, d.Qc, vals, wz, ww, lds, tid, BATCH_THREADS);
      }
    }
  }
}

}  // namespace

extern "C" LAM_API void lam_batch_destroy(lam_batch *b) {
  if (!b) return;
  for (lam_plan *p : b->plans) lam_plan_destroy(p);
  delete b;
}

extern "C" LAM_API lam_status lam_batch_create(int32_t n, const lam_laminate_desc *descs, int64_t wave_bytes,
                                               lam_batch **out) {
  if (!out || !descs || n < 1) return LAM_EINVAL;
  *out = nullptr;
  lam_batch *B = new (std::nothrow) lam_batch();
  if (!B) return LAM_EINVAL;
  B->n = n;
  int64_t cbytes = 0, ctot = 0, ttot = 0;
  for (int i = 0; i < n; ++i) {
    lam_plan *p = nullptr;
    lam_status st = lam_plan_create(&descs[i], &p);
    if (st != LAM_OK) {
      lam_batch_destroy(B);
      return st;
    }
    B->plans.push_back(p);
    // the fused kernel holds at most two set slots per scatter thread
    if (p->kron_nsc < 1 || p->kron_nsc > 2 || 3 * p->tile_k > BATCH_THREADS) {
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
  // work items per wave: the prep items, then the persistent queue
  for (int w = 0; w < B->n_waves; ++w) {
    const int f = B->wave_first[w], c = B->wave_count[w];
    B->wave_prep_off.push_back((int64_t)B->items.size());
    for (int i = f; i < f + c; ++i) {
      const lam_plan *p = B->plans[i];
      B->items.push_back(make_int4(i, ITEM_ROTATE, 0, 0));
      const int64_t nq = p->nnzz * std::max(p->kron_nsc, 1);
      for (int64_t j = 0; j < (nq + BATCH_THREADS - 1) / BATCH_THREADS; ++j)
        B->items.push_back(make_int4(i, ITEM_Q1D, (int)j, 0));
    }
    B->wave_prep_n.push_back((int)((int64_t)B->items.size() - B->wave_prep_off.back()));
    B->wave_items_off.push_back((int64_t)B->items.size());
    auto p2d = [&](int i) {
      const int np = (int)((B->plans[i]->nnz2 + BATCH_THREADS - 1) / BATCH_THREADS);
      for (int j = 0; j < np; ++j) B->items.push_back(make_int4(i, ITEM_P2D, j, 0));
    };
    auto kron = [&](int i) {
      const lam_plan *p = B->plans[i];
      for (int t = 0; t < p->n_tiles; ++t)
        for (int ch = 0; ch < p->n_chunks; ++ch) B->items.push_back(make_int4(i, ITEM_KRON, t, ch));
    };
    // 2D items run two laminates ahead of the scatter that needs them
    for (int i = f; i < std::min(f + 2, f + c); ++i) p2d(i);
    for (int i = f; i < f + c; ++i) {
      if (i + 2 < f + c) p2d(i + 2);
      kron(i);
    }
    B->wave_items_n.push_back((int)((int64_t)B->items.size() - B->wave_items_off.back()));
  }
  // batch workspace: tables | arena | Dev[n] | Meta[n] | items | counters
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
  B->counters_off = off;
  off = a256(off + (int64_t)sizeof(int) * (2 + n));
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
    devs[i] = lamdev::make_dev_split(p, base + b->const_off[i], base + b->arena_off + b->scratch_off[i]);
    meta[i].c_off = b->c_off[i];
    meta[i].t_off = b->t_off[i];
    meta[i].vals_off = b->vals_off[i];
    meta[i].n_p_items = (int)((p->nnz2 + BATCH_THREADS - 1) / BATCH_THREADS);
    meta[i].pad = 0;
  }
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      khz <= 0)
    return LAM_EHIP;
  b->wall_khz = khz;
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
  BatchArgs a;
  a.devs = reinterpret_cast<const Dev *>(base + b->devs_off);
  a.meta = reinterpret_cast<const Meta *>(base + b->meta_off);
  a.items = reinterpret_cast<const int4 *>(base + b->items_off) + b->wave_items_off[wave];
  a.n_items = b->wave_items_n[wave];
  a.counters = reinterpret_cast<int *>(base + b->counters_off);
  a.C_all = C_all;
  a.th_all = theta_all;
  a.vals = vals_wave;
  a.wait_ticks = (long long)b->wall_khz * LAM_BATCH_WAIT_MS;
  const int nc = 2 + b->n;
  hipLaunchKernelGGL(k_batch_reset, dim3((nc + 255) / 256), dim3(256), 0, s, a.counters, nc);
  void *prof = lam::profile_begin(3, stream);
  hipLaunchKernelGGL(k_batch_prep, dim3(b->wave_prep_n[wave]), dim3(BATCH_THREADS), 0, s, a,
                     reinterpret_cast<const int4 *>(base + b->items_off) + b->wave_prep_off[wave]);
  hipLaunchKernelGGL(k_batch, dim3(b->grid), dim3(BATCH_THREADS), (size_t)b->lds_bytes, s, a);
  lam::profile_end(prof, stream);
  return hipGetLastError() == hipSuccess ? LAM_OK : LAM_EHIP;
}

extern "C" LAM_API lam_status lam_batch_check(const lam_batch *b, const void *ws, int64_t ws_bytes, int32_t *error,
                                              void *stream) {
  if (!b || !ws || !error) return LAM_EINVAL;
  if (ws_bytes < b->total) return LAM_ESIZE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int v = 0;
  if (hipMemcpyAsync(&v, static_cast<const char *>(ws) + b->counters_off + sizeof(int), sizeof(int),
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LAM_EHIP;
  *error = v;
  return LAM_OK;
}
