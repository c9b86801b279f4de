// kp_dense.hip -- dense (code-indexed) accumulation of a Laurent product.
//
// Section 3.1: every pair of terms adds C_n * C_m at position n + m of a
// zero-initialised coefficient array indexed by code.  Section 4 observes that
// with sorted factors, blocks of consecutive terms write disjoint intervals of
// that array, so concurrent workers need no locks.  On gfx950 the array is cut
// into windows of S consecutive product codes; one workgroup owns a window in
// LDS (S * 8 bytes, up to 160 KB), finds by binary search over the sorted
// factors exactly the pairs whose code falls in the window, adds them with
// 64-bit LDS atomics (ds_add_u64 / ds_add_f64) and compacts the nonzero
// entries in code order.
//
// Work distribution.  Factor B is cut into tiles of 64 consecutive terms, one
// per lane of a wavefront; for a tile and a window the rows of A that can hit
// the window form one interval [i0, i1) (binary search on A's sorted codes),
// and a wavefront walks it with A's (code, coefficient) pair in scalar
// registers.  A planning pass counts these row visits per (window, tile);
// windows whose count exceeds an equal share of the total are split across
// several workgroups, which add their partial windows into an HBM array with
// device-scope atomics; the last of them to finish compacts the window.
//
// Launch sequence (one stream): plan_tiles -> plan_tasks -> zero_shared ->
// mul -> out_scan -> out_copy.
#include <climits>
#include <type_traits>

#include "kp_internal.h"

namespace kp {

namespace {

constexpr int PLAN_BLOCK = 256;
constexpr int64_t TASK_MIN_WORK = 512;   // row visits below which splitting a window does not pay

__device__ inline int64_t lower_bound(const int64_t* __restrict__ a, int64_t n, int64_t key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ inline int64_t readfirst64(int64_t v) {
  int32_t lo = __builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  int32_t hi = __builtin_amdgcn_readfirstlane((int32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Block-wide inclusive scan of one int64 per thread (any multiple of 64 threads).
template <int BS>
__device__ inline int64_t block_inclusive_scan(int64_t v, int64_t* s_wave, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    int64_t u = __shfl_up(v, off);
    if (lane >= off) v += u;
  }
  if (lane == 63) s_wave[wave] = v;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int w = 0; w < BS / 64; ++w) {
    int64_t x = s_wave[w];
    if (w < wave) before += x;
    all += x;
  }
  __syncthreads();
  *total = all;
  return v + before;
}

// ---------------------------------------------------------------- planning
// One workgroup per window: row visits of every B tile, inclusive prefix.
__global__ void __launch_bounds__(PLAN_BLOCK)
k_plan_tiles(int64_t S, int64_t ntiles, const int64_t* __restrict__ ak, int64_t na,
             const int64_t* __restrict__ bk, int64_t nb, int64_t* __restrict__ wt) {
  __shared__ int64_t s_wave[PLAN_BLOCK / 64];
  const int64_t w = blockIdx.x;
  const int64_t L = w * S;
  int64_t running = 0;
  for (int64_t base = 0; base < ntiles; base += PLAN_BLOCK) {
    const int64_t t = base + threadIdx.x;
    int64_t work = 0;
    if (t < ntiles) {
      const int64_t j0 = t * 64;
      const int64_t j1 = min(j0 + 64, nb) - 1;
      const int64_t i0 = lower_bound(ak, na, L - bk[j1]);
      const int64_t i1 = lower_bound(ak, na, L + S - bk[j0]);
      work = i1 - i0;
    }
    int64_t tot;
    int64_t inc = block_inclusive_scan<PLAN_BLOCK>(work, s_wave, &tot);
    if (t < ntiles) wt[w * ntiles + t] = running + inc;
    running += tot;
  }
}

// Single workgroup: split windows into tasks of about total / target row visits.
__global__ void __launch_bounds__(1024)
k_plan_tasks(int64_t nwin, int64_t ntiles, int64_t target, const int64_t* __restrict__ wt,
             int64_t* __restrict__ task_off, int32_t* __restrict__ pending,
             int64_t* __restrict__ wcount, Meta* meta) {
  __shared__ int64_t s_wave[16];
  int64_t sum = 0;
  for (int64_t w = threadIdx.x; w < nwin; w += 1024) sum += wt[w * ntiles + ntiles - 1];
  int64_t total;
  block_inclusive_scan<1024>(sum, s_wave, &total);
  int64_t T = (total + target - 1) / target;
  if (T < TASK_MIN_WORK) T = TASK_MIN_WORK;
  int64_t running = 0;
  for (int64_t base = 0; base < nwin; base += 1024) {
    const int64_t w = base + threadIdx.x;
    int64_t cnt = 0;
    if (w < nwin) {
      int64_t work = wt[w * ntiles + ntiles - 1];
      cnt = (work + T - 1) / T;
    }
    int64_t tot;
    int64_t inc = block_inclusive_scan<1024>(cnt, s_wave, &tot);
    if (w < nwin) {
      task_off[w] = running + inc - cnt;
      pending[w] = (int32_t)cnt;
      wcount[w] = 0;
    }
    running += tot;
  }
  if (threadIdx.x == 0) {
    task_off[nwin] = running;
    meta->ntasks = running;
  }
}

// Zero the HBM accumulator of every window shared by two or more tasks.
__global__ void __launch_bounds__(256)
k_zero_shared(int64_t S, const int64_t* __restrict__ task_off, int64_t* __restrict__ dense) {
  const int64_t w = blockIdx.x;
  if (task_off[w + 1] - task_off[w] < 2) return;
  int64_t* d = dense + w * S;
  for (int64_t i = threadIdx.x; i < S; i += 256) d[i] = 0;
}

// ------------------------------------------------------------ multiply
// Coefficient product.  MUL: 2 = both factors fit signed 24 bits (two
// full-rate 24-bit multiplies), 1 = both fit int32 (one 32x32->64 multiply),
// 0 = general int64 (wraps modulo 2^64), 3 = fp64.
template <typename T, int MUL>
__device__ inline T coef_mul_fixed(T a, T b) {
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

__device__ inline void lds_add(int64_t* p, int64_t v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}
__device__ inline void lds_add(double* p, double v) { unsafeAtomicAdd(p, v); }

__device__ inline void global_add(int64_t* p, int64_t v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}
__device__ inline void global_add(double* p, double v) { unsafeAtomicAdd(p, v); }

__device__ inline int64_t coherent_load(const int64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double coherent_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Ordered compaction of a window held in LDS: nonzero entries, ascending code.
template <typename T, int BS>
__device__ inline void compact_window(const T* win, int64_t S, int64_t L, int64_t* stage_k,
                                      T* stage_c, int64_t* count, int64_t* s_wave) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t run = 0;
  for (int64_t base = 0; base < S; base += BS) {
    const int64_t idx = base + threadIdx.x;
    T v = idx < S ? win[idx] : T(0);
    const bool f = v != T(0);
    const uint64_t m = __ballot(f);
    const int pre = __popcll(m & ((1ull << lane) - 1));
    if (lane == 0) s_wave[wave] = __popcll(m);
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) {
      int64_t x = s_wave[w];
      if (w < wave) before += x;
      all += x;
    }
    if (f) {
      const int64_t pos = run + before + pre;
      stage_k[pos] = L + idx;
      stage_c[pos] = v;
    }
    run += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = run;
}

// A wavefront's pass over rows [i0, i1) of A for one tile of B (one term per
// lane).  A's (code, coefficient) pairs are wavefront-uniform and live in
// scalar registers: eight at a time are fetched with two scalar loads and
// one wait (scalar loads return out of order, so a wave cannot overlap a
// later fetch with the use of an earlier one; other waves hide the latency).
// `apairs` must be readable 4 pairs past the last row (tail group).
template <int N>
struct PairsN {
  int64_t v[2 * N];
};

template <typename T, int MUL, bool WIDE>
__device__ inline void add_pair(T* win, int64_t a, int64_t craw, int64_t cj, uint32_t cj32,
                                uint32_t S32, bool valid, T cb) {
  bool hit;
  uint32_t slot;
  if (WIDE) {
    const int64_t d = a - cj;
    hit = (uint64_t)d < (uint64_t)S32;
    slot = (uint32_t)d;
  } else {
    slot = (uint32_t)a - cj32;
    hit = slot < S32;
  }
  if (valid && hit) {
    T ca;
    __builtin_memcpy(&ca, &craw, sizeof(T));
    lds_add(&win[slot], coef_mul_fixed<T, MUL>(ca, cb));
  }
}

template <typename T, int MUL, bool WIDE>
__device__ inline void rows_loop(T* win, const int64_t* __restrict__ apairs, int64_t i0, int64_t i1,
                                 int64_t cj, bool valid, T cb, int64_t S) {
  const uint32_t cj32 = (uint32_t)cj;
  const uint32_t S32 = (uint32_t)S;
  int64_t i = i0;
  for (; i + 8 <= i1; i += 8) {
    const PairsN<8> q = *reinterpret_cast<const PairsN<8>*>(apairs + 2 * i);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      add_pair<T, MUL, WIDE>(win, q.v[2 * u], q.v[2 * u + 1], cj, cj32, S32, valid, cb);
  }
  for (; i < i1; i += 4) {
    const PairsN<4> q = *reinterpret_cast<const PairsN<4>*>(apairs + 2 * i);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u < i1)
        add_pair<T, MUL, WIDE>(win, q.v[2 * u], q.v[2 * u + 1], cj, cj32, S32, valid, cb);
  }
}

template <typename T, bool WIDE>
__device__ inline void tile_rows(T* win, const int64_t* __restrict__ apairs, int64_t i0, int64_t i1,
                                 int64_t cj, bool valid, T cb, int64_t S, uint32_t narrow) {
  if (i0 >= i1) return;
  if constexpr (std::is_same<T, double>::value) {
    (void)narrow;
    rows_loop<T, 3, WIDE>(win, apairs, i0, i1, cj, valid, cb, S);
  } else {
    if (narrow & 2u)
      rows_loop<T, 2, WIDE>(win, apairs, i0, i1, cj, valid, cb, S);
    else if (narrow & 1u)
      rows_loop<T, 1, WIDE>(win, apairs, i0, i1, cj, valid, cb, S);
    else
      rows_loop<T, 0, WIDE>(win, apairs, i0, i1, cj, valid, cb, S);
  }
}

template <typename T, int BS>
__global__ void __launch_bounds__(BS)
k_dense_mul(int64_t S, int64_t nwin, int64_t ntiles, const Meta* __restrict__ meta,
            const int64_t* __restrict__ ak, const int64_t* __restrict__ apairs, int64_t na,
            const int64_t* __restrict__ bk, const T* __restrict__ bc, int64_t nb,
            const int64_t* __restrict__ wt, const int64_t* __restrict__ task_off,
            int32_t* __restrict__ pending, T* __restrict__ dense, int64_t* __restrict__ stage_k,
            T* __restrict__ stage_c, int64_t* __restrict__ wcount) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* win = reinterpret_cast<T*>(smem_raw);
  __shared__ int64_t s_wave[BS / 64];
  __shared__ int s_next;
  __shared__ int s_last;

  const int64_t task = blockIdx.x;
  if (task >= meta->ntasks) return;
  const uint32_t narrow = meta->narrow;

  // window of this task: last w with task_off[w] <= task
  int64_t lo = 0, hi = nwin;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (task_off[mid] <= task) lo = mid; else hi = mid;
  }
  const int64_t w = lo;
  const int64_t cnt = task_off[w + 1] - task_off[w];
  const int64_t k = task - task_off[w];
  const int64_t L = w * S;
  const int64_t* wtw = wt + w * ntiles;
  const int64_t tot = wtw[ntiles - 1];
  const int64_t lo_work = tot * k / cnt, hi_work = tot * (k + 1) / cnt;
  // tile t starts at prefix wtw[t-1] (0 for t = 0); take tiles starting in [lo_work, hi_work)
  const int64_t t_begin = lo_work == 0 ? 0 : min(ntiles, lower_bound(wtw, ntiles, lo_work) + 1);
  const int64_t t_end = hi_work == 0 ? 0 : min(ntiles, lower_bound(wtw, ntiles, hi_work) + 1);

  for (int64_t i = threadIdx.x; i < S; i += BS) win[i] = T(0);
  if (threadIdx.x == 0) s_next = (int)t_begin;
  __syncthreads();

  const int lane = threadIdx.x & 63;
  while (true) {
    int t = 0;
    if (lane == 0) t = atomicAdd(&s_next, 1);
    t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
    if (t >= t_end) break;
    const int64_t j0 = (int64_t)t * 64;
    const int64_t jl = min(j0 + 64, nb) - 1;
    const int64_t j = j0 + lane;
    const bool valid = j < nb;
    const int64_t bj = valid ? bk[j] : 0;
    const T cb = valid ? bc[j] : T(0);
    const int64_t bmin = readfirst64(bk[j0]), bmax = readfirst64(bk[jl]);
    const int64_t i0 = readfirst64(lower_bound(ak, na, L - bmax));
    const int64_t i1 = readfirst64(lower_bound(ak, na, L + S - bmin));
    const int64_t cj = L - bj;
    // d = a - cj is the slot of a pair in the window.  Over this tile's row
    // interval |d| < S + (bmax - bmin), so when that is below 2^31 the low
    // 32 bits decide the range test exactly.
    if (bmax - bmin < (int64_t)0x7fffffff - S)
      tile_rows<T, false>(win, apairs, i0, i1, cj, valid, cb, S, narrow);
    else
      tile_rows<T, true>(win, apairs, i0, i1, cj, valid, cb, S, narrow);
  }
  __syncthreads();

  if (cnt == 1) {
    compact_window<T, BS>(win, S, L, stage_k + L, stage_c + L, &wcount[w], s_wave);
    return;
  }
  // shared window: fold the partial sums into HBM, the last task compacts
  T* dw = dense + L;
  for (int64_t i = threadIdx.x; i < S; i += BS) {
    T v = win[i];
    if (v != T(0)) global_add(&dw[i], v);
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicSub(&pending[w], 1) == 1;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  for (int64_t i = threadIdx.x; i < S; i += BS) win[i] = coherent_load(&dw[i]);
  __syncthreads();
  compact_window<T, BS>(win, S, L, stage_k + L, stage_c + L, &wcount[w], s_wave);
}

// ------------------------------------------------------------ output
__global__ void __launch_bounds__(1024)
k_out_scan(int64_t nwin, const int64_t* __restrict__ wcount, int64_t* __restrict__ woff,
           Meta* meta) {
  __shared__ int64_t s_wave[16];
  int64_t running = 0;
  for (int64_t base = 0; base < nwin; base += 1024) {
    const int64_t w = base + threadIdx.x;
    const int64_t c = w < nwin ? wcount[w] : 0;
    int64_t tot;
    int64_t inc = block_inclusive_scan<1024>(c, s_wave, &tot);
    if (w < nwin) woff[w] = running + inc - c;
    running += tot;
  }
  if (threadIdx.x == 0) meta->out_count = running;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_out_copy(int64_t S, const Meta* __restrict__ meta, int64_t out_cap,
           const int64_t* __restrict__ wcount, const int64_t* __restrict__ woff,
           const int64_t* __restrict__ stage_k, const T* __restrict__ stage_c,
           int64_t* __restrict__ out_k, T* __restrict__ out_c) {
  if (meta->out_count > out_cap) return;
  const int64_t w = blockIdx.x;
  const int64_t n = wcount[w], off = woff[w];
  const int64_t* sk = stage_k + w * S;
  const T* sc = stage_c + w * S;
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    out_k[off + r] = sk[r];
    out_c[off + r] = sc[r];
  }
}

template <typename T>
hipError_t run_dense(const DensePlan& P, const DenseBufs& B, hipStream_t s) {
  const unsigned nwin = (unsigned)P.nwin;
  hipLaunchKernelGGL(k_plan_tiles, dim3(nwin), dim3(PLAN_BLOCK), 0, s, P.S, P.ntiles, B.ak, B.na,
                     B.bk, B.nb, B.wt);
  hipLaunchKernelGGL(k_plan_tasks, dim3(1), dim3(1024), 0, s, P.nwin, P.ntiles, P.target_tasks,
                     B.wt, B.task_off, B.pending, B.wcount, B.meta);
  hipLaunchKernelGGL(k_zero_shared, dim3(nwin), dim3(256), 0, s, P.S, B.task_off, (int64_t*)B.dense);
  const size_t lds = (size_t)P.S * sizeof(T);
  const T* bc = reinterpret_cast<const T*>(B.bc);
  T* dense = reinterpret_cast<T*>(B.dense);
  T* stage_c = reinterpret_cast<T*>(B.stage_c);
#define KP_DENSE_LAUNCH(BSZ)                                                                    \
  hipLaunchKernelGGL((k_dense_mul<T, BSZ>), dim3((unsigned)P.max_tasks), dim3(BSZ), lds, s, P.S, \
                     P.nwin, P.ntiles, B.meta, B.ak, B.apairs, B.na, B.bk, bc, B.nb, B.wt,      \
                     B.task_off, B.pending, dense, B.stage_k, stage_c, B.wcount)
  if (B.ev0) (void)hipEventRecord(B.ev0, s);
  if (P.block == 256)
    KP_DENSE_LAUNCH(256);
  else if (P.block == 512)
    KP_DENSE_LAUNCH(512);
  else
    KP_DENSE_LAUNCH(1024);
#undef KP_DENSE_LAUNCH
  if (B.ev1) (void)hipEventRecord(B.ev1, s);
  hipLaunchKernelGGL(k_out_scan, dim3(1), dim3(1024), 0, s, P.nwin, B.wcount, B.woff, B.meta);
  hipLaunchKernelGGL((k_out_copy<T>), dim3(nwin), dim3(256), 0, s, P.S, B.meta, B.out_cap, B.wcount,
                     B.woff, B.stage_k, stage_c, B.out_k, reinterpret_cast<T*>(B.out_c));
  return hipGetLastError();
}

template <typename T, int BS>
hipError_t set_lds_limit() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_mul<T, BS>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
}

}  // namespace

hipError_t launch_dense_laurent(const DensePlan& P, const DenseBufs& B, kp_dtype dt, hipStream_t s) {
  static bool attrs = false;
  if (!attrs) {
    hipError_t e = set_lds_limit<int64_t, 256>();
    if (e == hipSuccess) e = set_lds_limit<int64_t, 512>();
    if (e == hipSuccess) e = set_lds_limit<int64_t, 1024>();
    if (e == hipSuccess) e = set_lds_limit<double, 256>();
    if (e == hipSuccess) e = set_lds_limit<double, 512>();
    if (e == hipSuccess) e = set_lds_limit<double, 1024>();
    if (e != hipSuccess) return e;
    attrs = true;
  }
  return dt == KP_F64 ? run_dense<double>(P, B, s) : run_dense<int64_t>(P, B, s);
}

}  // namespace kp
