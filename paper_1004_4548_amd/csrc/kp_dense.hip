// kp_dense.hip -- dense (code-indexed) accumulation of a Laurent product.
//
// Section 3.1: every pair of terms adds C_n * C_m at position n + m of a
// zero-initialised coefficient array indexed by code; the factors are sorted
// by code so that products walk the array in order, and Section 4 notes that
// sorted blocks of the factors write disjoint intervals of it, so concurrent
// workers need no locks.  On gfx950 the array is cut into windows of
// consecutive product codes; one workgroup owns a window in LDS (up to 18432
// eight-byte slots), adds every pair whose code falls in it with 64-bit LDS
// atomics (ds_add_u64 / ds_add_f64) and compacts the nonzero slots in code
// order.
//
// Launches (one stream):
//  1. prep    -- two workgroups, one per factor: bucket sort by code (buckets
//                of 2^shift codes: LDS histogram, scan, scatter), A's bucket
//                start table, B's per-tile code min/max, coefficient-range
//                flags.
//  2. plan    -- one workgroup per window counts the row visits of every tile
//                of B; the last one to finish gives every window a number of
//                tasks proportional to its work.
//  3. mul     -- one workgroup per task.  Factor B is cut into tiles of 64
//                consecutive terms (one per lane); for a window [L, L+S) and a
//                tile with codes in [bmin, bmax] the rows of A that can land
//                in the window are those with codes in [L - bmax, L + S - bmin),
//                a run of buckets of A read off the bucket table in O(1); rows
//                with codes in [L - bmin, L + S - bmax) land in the window for
//                every lane and skip the range test.  A task takes a slice of
//                the window's tiles (equal work); wavefronts load 64 rows of A
//                at a time (the next 64 requested before the current ones are
//                used) and broadcast each row's code and coefficient to all
//                lanes with v_readlane.  A window with one task compacts its
//                nonzero slots straight from LDS; a window split into several
//                tasks writes each task's partial window to HBM.
//  4. combine -- one workgroup per chunk of a split window: sums the partial
//                windows and compacts the chunk.
//  5. scan    -- one workgroup: output offset of every chunk, result count.
//  6. copy    -- one workgroup per chunk: moves the chunk to its offset.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "kp_internal.h"

namespace kp {

namespace {

constexpr int PREP_BLOCK = 1024;
constexpr int PLAN_BLOCK = 256;
constexpr int PREP_UNROLL = 8;

__device__ __forceinline__ int64_t readfirst64(int64_t v) {
  int32_t lo = __builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  int32_t hi = __builtin_amdgcn_readfirstlane((int32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Block-wide exclusive scan of one int64 per thread; returns the exclusive
// prefix and writes the block total.  Two barriers.
template <int BS>
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* s_wave, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    int64_t u = __shfl_up(inc, off);
    if (lane >= off) inc += u;
  }
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < BS / 64; ++w) {
    int64_t x = s_wave[w];
    if (w < wave) before += x;
    all += x;
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

// Rows of A (bucket b holds codes [b << shift, (b+1) << shift)) that may hold
// codes in [lo, hi): the union of the buckets covering that interval.
__device__ __forceinline__ void rows_for(const int32_t* __restrict__ bstart, int shift, int64_t nbk,
                                int64_t lo, int64_t hi, int64_t* i0, int64_t* i1) {
  const int64_t maxcode = (nbk << shift) - 1;
  if (hi <= 0 || lo > maxcode || hi <= lo) {
    *i0 = *i1 = 0;
    return;
  }
  const int64_t b0 = (lo < 0 ? 0 : lo) >> shift;
  const int64_t b1 = ((hi - 1 > maxcode ? maxcode : hi - 1) >> shift) + 1;
  *i0 = bstart[b0];
  *i1 = bstart[b1];
}

// ------------------------------------------------------------------ prep
struct PrepSeg {
  const int64_t* keys;
  const int64_t* coef;    // 8-byte payload
  int64_t n;
  int shift;
  int64_t nbk;            // buckets (<= DENSE_MAX_BUCKETS)
  int64_t maxcode;        // largest code of the factor's box
  int64_t* out_keys;
  int64_t* out_coef;
  int32_t* rank;          // scratch [n]
  int32_t* bstart;        // [nbk + 1] (factor A only, else null)
  int64_t* tmin;          // [ceil(n/64)] (factor B only, else null)
  int64_t* tmax;
  int64_t* zero;          // array cleared by this workgroup (chunk counts), may be null
  int64_t nzero;
};
struct PrepArgs {
  PrepSeg seg[2];
  Meta* meta;
  int is_i64;
};

__global__ void __launch_bounds__(PREP_BLOCK) k_dense_prep(PrepArgs args) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int32_t* hist = reinterpret_cast<int32_t*>(smem_raw);
  __shared__ int64_t s_wave[PREP_BLOCK / 64];
  __shared__ uint32_t s_flags[PREP_BLOCK / 64];
  __shared__ uint32_t s_err[PREP_BLOCK / 64];
  const int which = blockIdx.x;
  const PrepSeg sg = args.seg[which];
  const int tid = threadIdx.x;
  const int64_t nbk = sg.nbk;
  const int64_t maxb = nbk - 1;

  if (which == 0 && tid == 0) {
    args.meta->plan_done = 0;
    args.meta->err = 0;
  }
  for (int64_t b = tid; b < nbk; b += PREP_BLOCK) hist[b] = 0;
  for (int64_t i = tid; i < sg.nzero; i += PREP_BLOCK) sg.zero[i] = 0;
  __syncthreads();
  uint32_t flags = 3u;   // bit0 fits int32, bit1 fits signed 24 bits
  uint32_t err = 0;
  // PREP_UNROLL elements per thread per round: all loads first, then the atomics
  for (int64_t base = 0; base < sg.n; base += PREP_BLOCK * PREP_UNROLL) {
    int64_t kk[PREP_UNROLL], cc[PREP_UNROLL];
#pragma unroll
    for (int u = 0; u < PREP_UNROLL; ++u) {
      const int64_t i = base + u * PREP_BLOCK + tid;
      kk[u] = i < sg.n ? sg.keys[i] : 0;
      cc[u] = (args.is_i64 && i < sg.n) ? sg.coef[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < PREP_UNROLL; ++u) {
      const int64_t i = base + u * PREP_BLOCK + tid;
      if (i >= sg.n) continue;
      const int64_t k = kk[u];
      int64_t b = k >> sg.shift;
      if (k < 0 || k > sg.maxcode) {   // a code outside the factor's box: flagged
        err |= ERR_RANGE;
        b = k < 0 ? 0 : min(b, maxb);
      }
      sg.rank[i] = atomicAdd(&hist[b], 1);
      const int64_t c = cc[u];
      if (c < INT_MIN || c > INT_MAX) flags &= ~1u;
      if (c < -(1 << 23) || c >= (1 << 23)) flags &= ~2u;
    }
  }
  __syncthreads();
  // exclusive scan of the histogram: each thread owns a contiguous run
  const int64_t per = (nbk + PREP_BLOCK - 1) / PREP_BLOCK;
  const int64_t b0 = min(nbk, tid * per), b1 = min(b0 + per, nbk);
  int64_t local = 0;
  for (int64_t b = b0; b < b1; ++b) local += hist[b];
  int64_t total;
  int64_t run = block_exclusive_scan<PREP_BLOCK>(local, s_wave, &total);
  for (int64_t b = b0; b < b1; ++b) {
    const int32_t c = hist[b];
    hist[b] = (int32_t)run;
    if (sg.bstart) sg.bstart[b] = (int32_t)run;
    run += c;
  }
  if (sg.bstart && tid == 0) sg.bstart[nbk] = (int32_t)sg.n;
  __syncthreads();
  for (int64_t base = 0; base < sg.n; base += PREP_BLOCK * PREP_UNROLL) {
    int64_t kk[PREP_UNROLL], cc[PREP_UNROLL];
    int32_t rr[PREP_UNROLL];
#pragma unroll
    for (int u = 0; u < PREP_UNROLL; ++u) {
      const int64_t i = base + u * PREP_BLOCK + tid;
      kk[u] = i < sg.n ? sg.keys[i] : 0;
      cc[u] = i < sg.n ? sg.coef[i] : 0;
      rr[u] = i < sg.n ? sg.rank[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < PREP_UNROLL; ++u) {
      const int64_t i = base + u * PREP_BLOCK + tid;
      if (i >= sg.n) continue;
      const int64_t k = kk[u];
      int64_t b = k >> sg.shift;
      b = k < 0 ? 0 : (b > maxb ? maxb : b);
      const int64_t pos = hist[b] + rr[u];
      sg.out_keys[pos] = k;
      sg.out_coef[pos] = cc[u];
    }
  }
  const uint32_t wf = wave_and(flags), we = wave_or(err);
  if ((tid & 63) == 0) {
    s_flags[tid >> 6] = wf;
    s_err[tid >> 6] = we;
  }
  __syncthreads();   // also orders the scattered keys before the tile pass
  if (tid == 0) {
    uint32_t f = 3u, e = 0;
    for (int w = 0; w < PREP_BLOCK / 64; ++w) {
      f &= s_flags[w];
      e |= s_err[w];
    }
    args.meta->seg_flags[which] = f;
    args.meta->seg_err[which] = e;
  }
  if (sg.tmin) {   // code range of every tile of 64 consecutive sorted terms
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t ntiles = (sg.n + 63) / 64;
    constexpr int NWP = PREP_BLOCK / 64;
    for (int64_t t0 = 0; t0 < ntiles; t0 += NWP * PREP_UNROLL) {
      int64_t kk[PREP_UNROLL];
#pragma unroll
      for (int u = 0; u < PREP_UNROLL; ++u) {
        const int64_t j = (t0 + u * NWP + wave) * 64 + lane;
        kk[u] = j < sg.n ? sg.out_keys[j] : LLONG_MAX;
      }
#pragma unroll
      for (int u = 0; u < PREP_UNROLL; ++u) {
        const int64_t t = t0 + u * NWP + wave;
        const int64_t j = t * 64 + lane;
        int64_t lo = kk[u], hi = j < sg.n ? kk[u] : LLONG_MIN;
        for (int off = 32; off > 0; off >>= 1) {
          lo = min(lo, __shfl_xor(lo, off));
          hi = max(hi, __shfl_xor(hi, off));
        }
        if (lane == 0 && t < ntiles) {
          sg.tmin[t] = lo;
          sg.tmax[t] = hi;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ plan
struct PlanArgs {
  int64_t S, nwin, ntiles, nkeys, target, min_work;
  const int32_t* bstart;
  int shiftA;
  int64_t nbkA;
  const int64_t* tmin;
  const int64_t* tmax;
  int64_t* wt;
  int64_t* task_off;
  int64_t* dense;     // [nwin * S] accumulator of windows split across tasks
  Meta* meta;
};

__global__ void __launch_bounds__(PLAN_BLOCK) k_dense_plan(PlanArgs P) {
  __shared__ int64_t s_wave[PLAN_BLOCK / 64];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int64_t L = w * P.S;
  const int64_t Sw = min(P.S, P.nkeys - L);
  int64_t running = 0;
  for (int64_t base = 0; base < P.ntiles; base += PLAN_BLOCK) {
    const int64_t t = base + tid;
    int64_t v = 0;
    if (t < P.ntiles) {
      int64_t i0, i1;
      rows_for(P.bstart, P.shiftA, P.nbkA, L - P.tmax[t], L + Sw - P.tmin[t], &i0, &i1);
      v = i1 - i0;
    }
    int64_t tot;
    const int64_t ex = block_exclusive_scan<PLAN_BLOCK>(v, s_wave, &tot);
    if (t < P.ntiles) P.wt[w * P.ntiles + t] = running + ex + v;
    running += tot;
  }
  // a window with more than min_work row visits may be split: clear its
  // HBM accumulator now (tasks of a split window add into it)
  if (running > P.min_work) {
    int64_t* d = P.dense + L;
    for (int64_t i = tid; i < Sw; i += PLAN_BLOCK) d[i] = 0;
  }
  if (tid == 0) {
    __threadfence();
    s_last = atomicAdd(&P.meta->plan_done, 1u) == (uint32_t)(P.nwin - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // last workgroup: tasks per window proportional to its work
  const int64_t per = (P.nwin + PLAN_BLOCK - 1) / PLAN_BLOCK;
  const int64_t w0 = min(P.nwin, tid * per), w1 = min(w0 + per, P.nwin);
  auto work_of = [&](int64_t u) {
    return __hip_atomic_load(&P.wt[u * P.ntiles + P.ntiles - 1], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  };
  int64_t local = 0;
  for (int64_t u = w0; u < w1; ++u) local += work_of(u);
  int64_t total;
  block_exclusive_scan<PLAN_BLOCK>(local, s_wave, &total);
  int64_t T = (total + P.target - 1) / P.target;
  if (T < P.min_work) T = P.min_work;
  // windows at or below min_work are never split (their accumulator was not cleared)
  auto tasks_of = [&](int64_t u) {
    const int64_t wk = work_of(u);
    return wk <= P.min_work ? (wk > 0 ? (int64_t)1 : (int64_t)0) : (wk + T - 1) / T;
  };
  int64_t ntask = 0;
  for (int64_t u = w0; u < w1; ++u) ntask += tasks_of(u);
  int64_t all;
  int64_t off = block_exclusive_scan<PLAN_BLOCK>(ntask, s_wave, &all);
  for (int64_t u = w0; u < w1; ++u) {
    P.task_off[u] = off;
    off += tasks_of(u);
  }
  if (tid == 0) {
    P.task_off[P.nwin] = all;
    P.meta->ntasks = all;
  }
}

// ------------------------------------------------------------------ multiply
// Coefficient product.  MUL: 2 = both factors fit signed 24 bits (two
// full-rate 24-bit multiplies), 1 = both fit int32 (one 32x32->64 multiply),
// 0 = general int64 (wraps modulo 2^64), 3 = fp64.
template <typename T, int MUL>
__device__ __forceinline__ T coef_mul_fixed(T a, T b) {
  if constexpr (MUL == 3) {
    return a * b;
  } else if constexpr (MUL == 2) {
    int32_t x = ((int32_t)a << 8) >> 8, y = ((int32_t)b << 8) >> 8;
    return (int64_t)x * (int64_t)y;
  } else if constexpr (MUL == 1) {
    return (int64_t)(int32_t)a * (int64_t)(int32_t)b;
  } else {
    return (int64_t)((uint64_t)a * (uint64_t)b);
  }
}

__device__ __forceinline__ void lds_add(int64_t* p, int64_t v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void lds_add(double* p, double v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ uint32_t rl(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

template <typename T, int MUL>
__device__ __forceinline__ T coef_of(uint32_t clo, uint32_t chi) {
  if constexpr (MUL == 1 || MUL == 2) {
    (void)chi;
    return (T)(int32_t)clo;
  } else {
    const uint64_t bits = ((uint64_t)chi << 32) | clo;
    T c;
    __builtin_memcpy(&c, &bits, sizeof(T));
    return c;
  }
}

// Row kinds: MODE 0 = every lane lands in the window (no test); 1 = byte
// offset test on 32 bits (|slot| < 2^28); 2 = full 64-bit test.
template <typename T, int MUL, int MODE>
__device__ __forceinline__ void add_row(T* win, uint32_t alo, uint32_t ahi, uint32_t clo,
                                        uint32_t chi, int64_t cj, uint32_t off8, uint32_t S8,
                                        bool valid, T cb) {
  char* base = reinterpret_cast<char*>(win);
  if constexpr (MODE == 0) {
    (void)ahi; (void)cj; (void)S8; (void)valid;
    const uint32_t rel = (alo << 3) + off8;
    lds_add(reinterpret_cast<T*>(base + rel), coef_mul_fixed<T, MUL>(coef_of<T, MUL>(clo, chi), cb));
  } else if constexpr (MODE == 1) {
    (void)ahi; (void)cj;
    const uint32_t rel = (alo << 3) + off8;
    if (valid && rel < S8)
      lds_add(reinterpret_cast<T*>(base + rel),
              coef_mul_fixed<T, MUL>(coef_of<T, MUL>(clo, chi), cb));
  } else {
    (void)off8;
    const int64_t a = (int64_t)(((uint64_t)ahi << 32) | alo);
    const int64_t d = a - cj;
    if (valid && (uint64_t)d < (uint64_t)(S8 >> 3))
      lds_add(&win[d], coef_mul_fixed<T, MUL>(coef_of<T, MUL>(clo, chi), cb));
  }
}

// Rows [i0, i1) of A against one tile of B (i0 < i1, wavefront-uniform).
// Lane l holds row base + l; the next 64 rows are requested before the
// current 64 are used.  Loads are unconditional (row indices are clamped to
// the last row) so that the wait before the broadcasts covers only the
// current rows.
template <typename T, int MUL, int MODE>
__device__ __forceinline__ void rows_loop(T* win, const int64_t* __restrict__ ak,
                                          const uint64_t* __restrict__ ac, int64_t i0, int64_t i1,
                                          int64_t cj, uint32_t off8, uint32_t S8, bool valid,
                                          T cb) {
  constexpr bool NARROW = MUL == 1 || MUL == 2;
  const int lane = threadIdx.x & 63;
  const int64_t last = i1 - 1;
  int64_t r = min(i0 + lane, last);
  uint64_t ka = (uint64_t)ak[r];
  uint64_t kc = ac[r];
  for (int64_t base = i0; base < i1; base += 64) {
    const int64_t rn = min(base + 64 + lane, last);
    const uint64_t nka = (uint64_t)ak[rn];
    const uint64_t nkc = ac[rn];
    const uint32_t alo = (uint32_t)ka, ahi = (uint32_t)(ka >> 32);
    const uint32_t clo = (uint32_t)kc, chi = (uint32_t)(kc >> 32);
    const int64_t cnt = i1 - base;
    if (cnt >= 64) {
#pragma unroll
      for (int u = 0; u < 64; ++u)
        add_row<T, MUL, MODE>(win, rl(alo, u), MODE == 2 ? rl(ahi, u) : 0u, rl(clo, u),
                              NARROW ? 0u : rl(chi, u), cj, off8, S8, valid, cb);
    } else {
      for (int u = 0; u < (int)cnt; ++u)
        add_row<T, MUL, MODE>(win, rl(alo, u), MODE == 2 ? rl(ahi, u) : 0u, rl(clo, u),
                              NARROW ? 0u : rl(chi, u), cj, off8, S8, valid, cb);
    }
    ka = nka;
    kc = nkc;
  }
}

// One tile: rows [i0, c0) and [c1, i1) with the range test, [c0, c1) without.
template <typename T, int MUL>
__device__ __forceinline__ void tile_mul(T* win, const int64_t* ak, const uint64_t* ac,
                                         int64_t i0, int64_t c0, int64_t c1, int64_t i1, bool wide,
                                         int64_t cj, uint32_t off8, uint32_t S8, bool valid,
                                         T cb) {
  if (wide) {
    rows_loop<T, MUL, 2>(win, ak, ac, i0, i1, cj, off8, S8, valid, cb);
    return;
  }
  if (c0 > i0) rows_loop<T, MUL, 1>(win, ak, ac, i0, c0, cj, off8, S8, valid, cb);
  if (c1 > c0) rows_loop<T, MUL, 0>(win, ak, ac, c0, c1, cj, off8, S8, valid, cb);
  if (i1 > c1) rows_loop<T, MUL, 1>(win, ak, ac, c1, i1, cj, off8, S8, valid, cb);
}

struct MulArgs {
  const Meta* meta;
  const int64_t* ak;
  const uint64_t* ac;     // A coefficients (8-byte words)
  const int32_t* bstart;
  int shiftA;
  int64_t nbkA;
  const int64_t* bk;
  const int64_t* bc;
  int64_t nb, ntiles, S, nwin, nkeys;
  const int64_t* tmin;
  const int64_t* tmax;
  const int64_t* wt;
  const int64_t* task_off;
  int64_t* dense;
  int64_t* stage_k;
  int64_t* stage_c;
  int64_t* ccount;
};

// first index in a[0, n) whose value is > key (a non-decreasing)
__device__ __forceinline__ int64_t upper_bound(const int64_t* __restrict__ a, int64_t n,
                                               int64_t key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// window of a task: last w with task_off[w] <= task
__device__ __forceinline__ int64_t window_of(const int64_t* __restrict__ task_off, int64_t nwin,
                                             int64_t task) {
  int64_t lo = 0, hi = nwin;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (task_off[mid] <= task) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void global_add(int64_t* p, int64_t v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void global_add(double* p, double v) { unsafeAtomicAdd(p, v); }

constexpr int64_t ITEM_ROWS = 128;   // rows of A per work item

// A task owns the row visits [lo, hi) of its window, in the order (tile,
// row).  They are cut into items of at most ITEM_ROWS rows of one tile,
// listed in LDS and taken by wavefronts one at a time.
template <typename T, int BS>
__global__ void __launch_bounds__(BS) k_dense_mul(MulArgs M) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* win = reinterpret_cast<T*>(smem_raw);
  __shared__ int32_t s_tile[DENSE_MAX_TILES_LDS];
  __shared__ int32_t s_r0[DENSE_MAX_TILES_LDS];
  __shared__ int32_t s_r1[DENSE_MAX_TILES_LDS];
  __shared__ int64_t s_wave[BS / 64];
  __shared__ int s_next;

  const int64_t task = blockIdx.x;
  if (task >= M.meta->ntasks) return;
  const int64_t w = window_of(M.task_off, M.nwin, task);
  const int64_t k = M.task_off[w + 1] - M.task_off[w];
  const int64_t p = task - M.task_off[w];
  const int64_t L = w * M.S;
  const int64_t Sw = min(M.S, M.nkeys - L);
  const int64_t* wtw = M.wt + w * M.ntiles;
  const int64_t W = wtw[M.ntiles - 1];
  const int64_t lo = W * p / k, hi = W * (p + 1) / k;
  // tiles overlapping [lo, hi): tile t covers [wtw[t-1], wtw[t])
  const int64_t t_begin = upper_bound(wtw, M.ntiles, lo);
  const int64_t t_end = min(M.ntiles, upper_bound(wtw, M.ntiles, hi - 1) + 1);
  const uint32_t narrow = M.meta->seg_flags[0] & M.meta->seg_flags[1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T* bc = reinterpret_cast<const T*>(M.bc);
  const uint32_t S8 = (uint32_t)(Sw * 8);
  const int64_t bw = (int64_t)1 << M.shiftA;

  for (int64_t i = tid; i < Sw; i += BS) win[i] = T(0);
  int64_t t0 = t_begin;
  while (t0 < t_end) {
    // list items of tiles [t0, t1) until the LDS list would overflow
    const int64_t t1 = min(t_end, t0 + BS);
    const int64_t t = t0 + tid;
    int64_t r0 = 0, r1 = 0;
    if (t < t1) {
      int64_t i0, i1;
      rows_for(M.bstart, M.shiftA, M.nbkA, L - M.tmax[t], L + Sw - M.tmin[t], &i0, &i1);
      const int64_t s0 = t == 0 ? 0 : wtw[t - 1];
      r0 = i0 + max((int64_t)0, lo - s0);
      r1 = i0 + min(i1 - i0, hi - s0);
      if (r1 < r0) r1 = r0;
    }
    // at most 256 items per tile (longer tiles get longer items), so the
    // first tile of a round always fits the list
    const int64_t irows = max(ITEM_ROWS, (r1 - r0 + 255) / 256);
    const int64_t nit = (r1 - r0 + irows - 1) / irows;
    int64_t total;
    const int64_t pos = block_exclusive_scan<BS>(nit, s_wave, &total);
    // tiles whose items fit the list form a prefix of [t0, t1)
    const bool fits = t < t1 && pos + nit <= DENSE_MAX_TILES_LDS;
    if (fits)
      for (int64_t q = 0; q < nit; ++q) {
        s_tile[pos + q] = (int32_t)t;
        s_r0[pos + q] = (int32_t)(r0 + q * irows);
        s_r1[pos + q] = (int32_t)min(r1, r0 + (q + 1) * irows);
      }
    int64_t nitems;
    block_exclusive_scan<BS>(fits ? nit : 0, s_wave, &nitems);
    const uint64_t bal = __ballot(!fits && t < t1);
    if (lane == 0) s_wave[wave] = bal ? (int64_t)(wave * 64 + __ffsll((long long)bal) - 1) : BS;
    if (tid == 0) s_next = 0;
    __syncthreads();
    int64_t nlisted = BS;   // tiles listed this round
    for (int u = 0; u < BS / 64; ++u) nlisted = min(nlisted, s_wave[u]);
    // items: wavefronts take them dynamically
    while (true) {
      int e = 0;
      if (lane == 0) e = atomicAdd(&s_next, 1);
      e = __builtin_amdgcn_readfirstlane(__shfl(e, 0));
      if (e >= nitems) break;
      const int64_t tt = __builtin_amdgcn_readfirstlane(s_tile[e]);
      const int64_t a0 = __builtin_amdgcn_readfirstlane(s_r0[e]);
      const int64_t a1 = __builtin_amdgcn_readfirstlane(s_r1[e]);
      const int64_t j = tt * 64 + lane;
      const bool full = tt * 64 + 63 < M.nb;
      const bool valid = j < M.nb;
      const int64_t bj = valid ? M.bk[j] : 0;
      const T cb = valid ? bc[j] : T(0);
      const int64_t bmin = readfirst64(M.tmin[tt]), bmax = readfirst64(M.tmax[tt]);
      const int64_t cj = L - bj;
      const uint32_t off8 = (uint32_t)((uint64_t)(bj - L) << 3);
      // rows whose bucket lies inside [L - bmin, L + Sw - bmax) hit for every lane
      int64_t c0 = a0, c1 = a0;
      const int64_t clo = L - bmin, chi = L + Sw - bmax;
      if (full && chi > clo) {
        const int64_t b0 = (max(clo, (int64_t)0) + bw - 1) >> M.shiftA;
        const int64_t b1 = min(chi >> M.shiftA, M.nbkA);
        if (b1 > b0) {
          c0 = min(a1, max(a0, (int64_t)M.bstart[b0]));
          c1 = max(c0, min(a1, (int64_t)M.bstart[b1]));
        }
      }
      // byte offsets of the range test fit 32 bits while |slot| < 2^28
      const bool wide = (bmax - bmin) + Sw + bw >= ((int64_t)1 << 28);
      if constexpr (std::is_same<T, double>::value) {
        tile_mul<T, 3>(win, M.ak, M.ac, a0, c0, c1, a1, wide, cj, off8, S8, valid, cb);
      } else {
        if (narrow & 2u)
          tile_mul<T, 2>(win, M.ak, M.ac, a0, c0, c1, a1, wide, cj, off8, S8, valid, cb);
        else if (narrow & 1u)
          tile_mul<T, 1>(win, M.ak, M.ac, a0, c0, c1, a1, wide, cj, off8, S8, valid, cb);
        else
          tile_mul<T, 0>(win, M.ak, M.ac, a0, c0, c1, a1, wide, cj, off8, S8, valid, cb);
      }
    }
    __syncthreads();
    t0 += nlisted;
  }

  if (k > 1) {   // split window: add this task's nonzero slots into HBM
    T* d = reinterpret_cast<T*>(M.dense) + L;
    for (int64_t i = tid; i < Sw; i += BS) {
      const T v = win[i];
      if (v != T(0)) global_add(&d[i], v);
    }
    return;
  }
  // ordered compaction, one wavefront per chunk of the window
  constexpr int NW = BS / 64;
  const int64_t nch = (Sw + DENSE_CHUNK - 1) / DENSE_CHUNK;
  const uint64_t lt = (1ull << lane) - 1;
  for (int64_t c = wave; c < nch; c += NW) {
    const int64_t s0 = c * DENSE_CHUNK, s1 = min(Sw, s0 + DENSE_CHUNK);
    const int64_t gc = L / DENSE_CHUNK + c;
    int64_t* sk = M.stage_k + gc * DENSE_CHUNK;
    T* sc = reinterpret_cast<T*>(M.stage_c) + gc * DENSE_CHUNK;
    int64_t off = 0;
    for (int64_t b = s0; b < s1; b += 64) {
      const int64_t i = b + lane;
      const T v = i < s1 ? win[i] : T(0);
      const bool f = v != T(0);
      const uint64_t m = __ballot(f);
      if (f) {
        const int64_t q = off + __popcll(m & lt);
        sk[q] = L + i;
        sc[q] = v;
      }
      off += __popcll(m);
    }
    if (lane == 0) M.ccount[gc] = off;
  }
}

// ------------------------------------------------------------------ split windows
struct CombineArgs {
  const Meta* meta;
  const int64_t* task_off;
  int64_t nwin, S, nkeys;
  const int64_t* dense;
  int64_t* stage_k;
  int64_t* stage_c;
  int64_t* ccount;
};

constexpr int COMBINE_BLOCK = 256;
constexpr int COMBINE_PER = DENSE_CHUNK / COMBINE_BLOCK;   // slots per thread

// One workgroup per chunk of a window split across tasks: ordered compaction
// of the chunk's accumulated slots.
template <typename T>
__global__ void __launch_bounds__(COMBINE_BLOCK) k_dense_combine(CombineArgs C) {
  __shared__ int64_t s_wave[COMBINE_BLOCK / 64];
  const int64_t cpw = C.S / DENSE_CHUNK;
  const int64_t w = blockIdx.x / cpw, c = blockIdx.x - w * cpw;
  if (C.task_off[w + 1] - C.task_off[w] < 2) return;
  const int64_t L = w * C.S;
  const int64_t Sw = min(C.S, C.nkeys - L);
  const int64_t s0 = c * DENSE_CHUNK;
  if (s0 >= Sw) return;
  const int64_t s1 = min(Sw, s0 + DENSE_CHUNK);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* d = reinterpret_cast<const T*>(C.dense) + L;
  // wave owns the contiguous slots [s0 + wave * 512, +512), lane-strided
  T v[COMBINE_PER];
  uint64_t ball[COMBINE_PER];
  int64_t cnt = 0;
#pragma unroll
  for (int r = 0; r < COMBINE_PER; ++r) {
    const int64_t i = s0 + wave * (64 * COMBINE_PER) + r * 64 + lane;
    v[r] = i < s1 ? d[i] : T(0);
  }
#pragma unroll
  for (int r = 0; r < COMBINE_PER; ++r) {
    ball[r] = __ballot(v[r] != T(0));
    cnt += __popcll(ball[r]);
  }
  if (lane == 0) s_wave[wave] = cnt;
  __syncthreads();
  int64_t off = 0, all = 0;
#pragma unroll
  for (int u = 0; u < COMBINE_BLOCK / 64; ++u) {
    if (u < wave) off += s_wave[u];
    all += s_wave[u];
  }
  const int64_t gc = L / DENSE_CHUNK + c;
  int64_t* sk = C.stage_k + gc * DENSE_CHUNK;
  T* sc = reinterpret_cast<T*>(C.stage_c) + gc * DENSE_CHUNK;
  const uint64_t lt = (1ull << lane) - 1;
#pragma unroll
  for (int r = 0; r < COMBINE_PER; ++r) {
    if (ball[r] & (1ull << lane)) {
      const int64_t q = off + __popcll(ball[r] & lt);
      sk[q] = L + s0 + wave * (64 * COMBINE_PER) + r * 64 + lane;
      sc[q] = v[r];
    }
    off += __popcll(ball[r]);
  }
  if (threadIdx.x == 0) C.ccount[gc] = all;
}

// ------------------------------------------------------------------ output
struct ScanArgs {
  const Meta* meta;
  int64_t nchunk, out_cap;
  const int64_t* ccount;
  int64_t* coff;
  int64_t* out_n;
  uint32_t* ctx_err;
};

__global__ void __launch_bounds__(1024) k_dense_scan(ScanArgs A) {
  __shared__ int64_t s_wave[16];
  const int64_t per = (A.nchunk + 1023) / 1024;
  const int64_t c0 = min(A.nchunk, (int64_t)threadIdx.x * per), c1 = min(c0 + per, A.nchunk);
  int64_t local = 0;
  for (int64_t c = c0; c < c1; ++c) local += A.ccount[c];
  int64_t total;
  int64_t run = block_exclusive_scan<1024>(local, s_wave, &total);
  for (int64_t c = c0; c < c1; ++c) {
    A.coff[c] = run;
    run += A.ccount[c];
  }
  if (threadIdx.x == 0) {
    uint32_t e = A.meta->err | A.meta->seg_err[0] | A.meta->seg_err[1];
    if (total > A.out_cap) e |= ERR_CAPACITY;
    if (e) {
      atomicOr(A.ctx_err, e);
      *A.out_n = -(int64_t)first_error(e);
    } else {
      *A.out_n = total;
    }
  }
}

struct CopyArgs {
  int64_t out_cap;
  const int64_t* ccount;
  const int64_t* coff;
  const int64_t* stage_k;
  const int64_t* stage_c;
  int64_t* out_k;
  int64_t* out_c;
};

__global__ void __launch_bounds__(256) k_dense_copy(CopyArgs C) {
  const int64_t c = blockIdx.x;
  const int64_t n = C.ccount[c], off = C.coff[c];
  const int64_t* sk = C.stage_k + c * DENSE_CHUNK;
  const int64_t* sc = C.stage_c + c * DENSE_CHUNK;
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    const int64_t q = off + r;
    if (q < C.out_cap) {
      C.out_k[q] = sk[r];
      C.out_c[q] = sc[r];
    }
  }
}

template <typename T, int BS>
hipError_t set_lds_limit() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_mul<T, BS>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)DENSE_LDS_BYTES);
}

}  // namespace

int dense_bucket_shift(int64_t maxcode) {
  int s = 0;
  while (((maxcode >> s) + 1) > DENSE_MAX_BUCKETS) ++s;
  return s;
}

hipError_t launch_dense_laurent(const DensePlan& P, const DenseBufs& B, kp_dtype dt, hipStream_t s) {
  static bool attrs = false;
  if (!attrs) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_prep),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(DENSE_MAX_BUCKETS * 4));
    if (e == hipSuccess) e = set_lds_limit<int64_t, 256>();
    if (e == hipSuccess) e = set_lds_limit<int64_t, 512>();
    if (e == hipSuccess) e = set_lds_limit<int64_t, 1024>();
    if (e == hipSuccess) e = set_lds_limit<double, 256>();
    if (e == hipSuccess) e = set_lds_limit<double, 512>();
    if (e == hipSuccess) e = set_lds_limit<double, 1024>();
    if (e != hipSuccess) return e;
    attrs = true;
  }
  PrepArgs pa{};
  pa.seg[0] = PrepSeg{B.a_keys_in, B.a_coef_in, B.na, P.shiftA, P.nbkA, P.maxcodeA, B.ak, B.ac,
                      B.rank_a, B.bstart, nullptr, nullptr, nullptr, 0};
  pa.seg[1] = PrepSeg{B.b_keys_in, B.b_coef_in, B.nb, P.shiftB, P.nbkB, P.maxcodeB, B.bk, B.bc,
                      B.rank_b, nullptr, B.tmin, B.tmax, B.ccount, P.nchunk};
  pa.meta = B.meta;
  pa.is_i64 = dt == KP_I64;
  const size_t hist_bytes = (size_t)std::max(P.nbkA, P.nbkB) * 4;
  hipLaunchKernelGGL(k_dense_prep, dim3(2), dim3(PREP_BLOCK), hist_bytes, s, pa);

  PlanArgs pl{P.S, P.nwin, P.ntiles, P.nkeys, P.target_tasks, P.min_work, B.bstart, P.shiftA,
              P.nbkA, B.tmin, B.tmax, B.wt, B.task_off, B.dense, B.meta};
  hipLaunchKernelGGL(k_dense_plan, dim3((unsigned)P.nwin), dim3(PLAN_BLOCK), 0, s, pl);

  MulArgs ma{B.meta, B.ak, reinterpret_cast<const uint64_t*>(B.ac), B.bstart, P.shiftA, P.nbkA,
             B.bk, B.bc, B.nb, P.ntiles, P.S, P.nwin, P.nkeys, B.tmin, B.tmax, B.wt, B.task_off,
             B.dense, B.stage_k, B.stage_c, B.ccount};
  const size_t lds = (size_t)P.S * 8;
  const unsigned grid = (unsigned)P.max_tasks;
  if (B.ev0) (void)hipEventRecord(B.ev0, s);
#define KP_DENSE_LAUNCH(TT, BSZ) \
  hipLaunchKernelGGL((k_dense_mul<TT, BSZ>), dim3(grid), dim3(BSZ), lds, s, ma)
  if (dt == KP_F64) {
    if (P.block == 256) KP_DENSE_LAUNCH(double, 256);
    else if (P.block == 512) KP_DENSE_LAUNCH(double, 512);
    else KP_DENSE_LAUNCH(double, 1024);
  } else {
    if (P.block == 256) KP_DENSE_LAUNCH(int64_t, 256);
    else if (P.block == 512) KP_DENSE_LAUNCH(int64_t, 512);
    else KP_DENSE_LAUNCH(int64_t, 1024);
  }
#undef KP_DENSE_LAUNCH
  if (B.ev1) (void)hipEventRecord(B.ev1, s);

  CombineArgs cb{B.meta, B.task_off, P.nwin, P.S, P.nkeys, B.dense, B.stage_k, B.stage_c,
                 B.ccount};
  const unsigned cgrid = (unsigned)(P.nwin * (P.S / DENSE_CHUNK));
  if (dt == KP_F64)
    hipLaunchKernelGGL(k_dense_combine<double>, dim3(cgrid), dim3(COMBINE_BLOCK), 0, s, cb);
  else
    hipLaunchKernelGGL(k_dense_combine<int64_t>, dim3(cgrid), dim3(COMBINE_BLOCK), 0, s, cb);

  ScanArgs sa{B.meta, P.nchunk, B.out_cap, B.ccount, B.coff, B.out_n, B.ctx_err};
  hipLaunchKernelGGL(k_dense_scan, dim3(1), dim3(1024), 0, s, sa);
  CopyArgs ca{B.out_cap, B.ccount, B.coff, B.stage_k, B.stage_c, B.out_k,
              reinterpret_cast<int64_t*>(B.out_c)};
  hipLaunchKernelGGL(k_dense_copy, dim3((unsigned)P.nchunk), dim3(256), 0, s, ca);
  return hipGetLastError();
}

}  // namespace kp
