// kp_pack.hip -- many whole Laurent products in one fixed sequence of
// persistent launches.
//
// A pack keeps the products of a batch in a device task table.  Each stage is
// one launch of a fixed grid whose workgroups walk the units of every task
// (a unit is a slice of one task's work: terms to encode, table words to
// clear, a block of term pairs, a block of table slots); unit u belongs to the
// task whose prefix of units covers it.  The kernels read nothing but the
// table, so the sequence (the table's upload included) can be captured once
// into a HIP graph and replayed for every batch, whatever its products.
//
// Each product is the schoolbook sum of Section 3 over Kronecker codes
// (Section 2), accumulated in a table of its own in device memory: indexed by
// code when the key space is small (the dense array of Section 3.1), else an
// open-addressing hash table keyed by code, with a compare-and-swap on the key
// and an atomic add on the coefficient (Section 3.2).  Nonzero sums are
// compacted by wavefront ballots and decoded to exponents on the way out, and
// each task's count is posted to pinned host memory.

#include <climits>

#include "kp_internal.h"

namespace kp {

namespace {

constexpr int PACK_BOX_BLOCK = 1024;
constexpr int PACK_SLOTS_PER_THREAD = 8;
constexpr int PACK_CMP_SLOTS = PACK_BLOCK * PACK_SLOTS_PER_THREAD;
constexpr uint64_t GOLD = 0x9E3779B97F4A7C15ull;   // 2^64 / golden ratio (Fibonacci hashing)

struct PackView {
  PackHeader* h;
  const int64_t* pre_prep;
  const int64_t* pre_mul;
  const int64_t* pre_cmp;
  PackTask* tasks;
};

__device__ __forceinline__ PackView view(void* table) {
  PackView v;
  v.h = static_cast<PackHeader*>(table);
  const int m = v.h->max_tasks;
  int64_t* pre = reinterpret_cast<int64_t*>(static_cast<char*>(table) + sizeof(PackHeader));
  v.pre_prep = pre;
  v.pre_mul = pre + (m + 1);
  v.pre_cmp = pre + 2 * (m + 1);
  v.tasks = reinterpret_cast<PackTask*>(pre + 3 * (m + 1));
  return v;
}

// The task of unit u: the last k with pre[k] <= u (pre ascending, pre[0] = 0).
__device__ __forceinline__ int task_of(const int64_t* pre, int n, int64_t u) {
  int a = 0, z = n;
  while (z - a > 1) {
    const int m = (a + z) >> 1;
    if (pre[m] <= u) a = m;
    else z = m;
  }
  return a;
}

// ------------------------------------------------------------ boxes
// One workgroup per array: per-variable minimum and maximum, posted as tagged
// words (side 0 the minima, side 1 the maxima) to host-mapped memory.

__global__ void __launch_bounds__(PACK_BOX_BLOCK)
k_pack_boxes(const int32_t* const* vals, const int64_t* ns, const int32_t* nvs, uint64_t* post,
             uint64_t seq) {
  __shared__ int32_t smin[KP_MAX_VARS][PACK_BOX_BLOCK / 64];
  __shared__ int32_t smax[KP_MAX_VARS][PACK_BOX_BLOCK / 64];
  const int g = blockIdx.x;
  const int64_t n = ns[g];
  const int32_t nv = nvs[g];
  const int32_t* __restrict__ x = vals[g];
  int32_t lo[KP_MAX_VARS], hi[KP_MAX_VARS];
#pragma unroll
  for (int v = 0; v < KP_MAX_VARS; ++v) {
    lo[v] = INT_MAX;
    hi[v] = INT_MIN;
  }
  // rows, one per thread at a time (each row's nv words)
  for (int64_t r = threadIdx.x; r < n; r += PACK_BOX_BLOCK) {
#pragma unroll
    for (int v = 0; v < KP_MAX_VARS; ++v)
      if (v < nv) {
        const int32_t e = x[r * nv + v];
        lo[v] = min(lo[v], e);
        hi[v] = max(hi[v], e);
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < KP_MAX_VARS; ++v) {
    if (v >= nv) break;
    int32_t a = lo[v], b = hi[v];
    for (int off = 32; off > 0; off >>= 1) {
      a = min(a, __shfl_xor(a, off));
      b = max(b, __shfl_xor(b, off));
    }
    if (lane == 0) {
      smin[v][wave] = a;
      smax[v][wave] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * KP_MAX_VARS) {
    const int v = threadIdx.x % KP_MAX_VARS;
    const bool is_max = threadIdx.x >= KP_MAX_VARS;
    if (v < nv) {
      int32_t r = is_max ? INT_MIN : INT_MAX;
      for (int w = 0; w < PACK_BOX_BLOCK / 64; ++w)
        r = is_max ? max(r, smax[v][w]) : min(r, smin[v][w]);
      const uint64_t word = ((uint64_t)(uint32_t)seq << 32) | (uint32_t)r;
      __hip_atomic_store(&post[(size_t)g * 2 * KP_MAX_VARS + threadIdx.x], word, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// ------------------------------------------------------------ prep
// Units of a task: its rows of A and of B to encode (PACK_BLOCK each), then
// its table words to clear (4 * PACK_BLOCK each, at least one unit); the first
// clearing unit also resets the task's result counter.
__global__ void __launch_bounds__(PACK_BLOCK) k_pack_prep(void* table) {
  const PackView P = view(table);
  const int nt = P.h->ntasks;
  const int64_t total = P.pre_prep[nt];
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int k = task_of(P.pre_prep, nt, u);
    const PackTask& T = P.tasks[k];
    int64_t l = u - P.pre_prep[k];
    const int64_t ea = (T.na + PACK_BLOCK - 1) / PACK_BLOCK;
    const int64_t eb = (T.nb + PACK_BLOCK - 1) / PACK_BLOCK;
    if (l < ea + eb) {
      const bool isb = l >= ea;
      const int64_t r = (isb ? l - ea : l) * PACK_BLOCK + threadIdx.x;
      const int64_t n = isb ? T.nb : T.na;
      if (r < n) {
        const DevLayout& L = isb ? T.lb : T.la;
        const int32_t* x = (isb ? T.bx : T.ax) + r * L.nx;
        int32_t e[KP_MAX_VARS];
        for (int v = 0; v < L.nx; ++v) e[v] = x[v];
        int64_t kx = 0, ky = 0;
        const uint32_t bad = encode_term(L, e, nullptr, 0, &kx, &ky);
        if (bad) atomicOr(&P.h->err, bad);
        (isb ? T.bk : T.ak)[r] = kx;
      }
    } else {
      l -= ea + eb;
      const int64_t words = T.direct ? T.slots : 2 * T.slots;
      const int64_t w0 = l * 4 * PACK_BLOCK + threadIdx.x;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t w = w0 + (int64_t)q * PACK_BLOCK;
        if (w < words) T.table[w] = 0;
      }
      if (l == 0 && threadIdx.x == 0) *T.count = 0;
    }
  }
}

// ------------------------------------------------------------ multiply
__device__ __forceinline__ void add_value(uint64_t* p, bool f64, uint64_t bits) {
  if (f64) {
    double v;
    __builtin_memcpy(&v, &bits, 8);
    atomicAdd(reinterpret_cast<double*>(p), v);
  } else {
    atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)bits);
  }
}

// Units of a task: (block of `rows` rows of A, block of PACK_BLOCK terms of B);
// a thread takes one term of B against the block's rows (wavefront-uniform
// loads of A).  Each product is added at its code: directly, or in the hash
// table (linear probing from the code's Fibonacci hash).
__global__ void __launch_bounds__(PACK_BLOCK) k_pack_mul(void* table) {
  const PackView P = view(table);
  const int nt = P.h->ntasks;
  const int64_t total = P.pre_mul[nt];
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int k = task_of(P.pre_mul, nt, u);
    const PackTask& T = P.tasks[k];
    const int64_t l = u - P.pre_mul[k];
    const int64_t rb = l / T.bblocks, bb = l - rb * T.bblocks;
    const int64_t j = bb * PACK_BLOCK + threadIdx.x;
    if (j >= T.nb) continue;
    const int64_t kb = T.bk[j];
    const uint64_t cb = static_cast<const uint64_t*>(T.bc)[j];
    const int64_t i0 = rb * T.rows, i1 = min(T.na, i0 + T.rows);
    const bool f64 = T.f64 != 0;
    const uint64_t* ac = static_cast<const uint64_t*>(T.ac);
    const uint64_t mask = (uint64_t)T.slots - 1;
    const int shift = T.direct ? 0 : 64 - __builtin_ctzll((unsigned long long)T.slots);
    for (int64_t i = i0; i < i1; ++i) {
      const int64_t c = T.ak[i] + kb;
      uint64_t bits;
      if (f64) {
        double x, y;
        const uint64_t xa = ac[i];
        __builtin_memcpy(&x, &xa, 8);
        __builtin_memcpy(&y, &cb, 8);
        const double v = x * y;
        __builtin_memcpy(&bits, &v, 8);
      } else {
        bits = ac[i] * cb;   // wraps modulo 2^64
      }
      if (T.direct) {
        // codes lie in [0, slots) when the factors lie in their planned boxes
        if ((uint64_t)c < (uint64_t)T.slots) add_value(T.table + c, f64, bits);
        else atomicOr(&P.h->err, ERR_RANGE);
        continue;
      }
      const unsigned long long key = (unsigned long long)c + 1;
      uint64_t s = ((uint64_t)c * GOLD) >> shift;
      int64_t q = 0;
      for (; q < T.slots; ++q) {   // the table holds at least twice the task's terms
        unsigned long long* ks = reinterpret_cast<unsigned long long*>(T.table + 2 * s);
        unsigned long long cur = __hip_atomic_load(ks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == 0) {
          cur = atomicCAS(ks, 0ull, key);
          if (cur == 0) cur = key;
        }
        if (cur == key) {
          add_value(T.table + 2 * s + 1, f64, bits);
          break;
        }
        s = (s + 1) & mask;
      }
      if (q == T.slots) atomicOr(&P.h->err, ERR_CAPACITY);
    }
  }
}

// ------------------------------------------------------------ compaction
// Units of a task: blocks of PACK_CMP_SLOTS table slots.  Nonzero sums are
// compacted by ballots, placed after one atomic on the task's counter, and
// written as decoded exponents and coefficients.
__global__ void __launch_bounds__(PACK_BLOCK) k_pack_compact(void* table) {
  __shared__ int64_t s_wave[PACK_BLOCK / 64];
  __shared__ int64_t s_base;
  const PackView P = view(table);
  const int nt = P.h->ntasks;
  const int64_t total = P.pre_cmp[nt];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int k = task_of(P.pre_cmp, nt, u);
    const PackTask& T = P.tasks[k];
    const int64_t s0 = (u - P.pre_cmp[k]) * PACK_CMP_SLOTS;
    int64_t code[PACK_SLOTS_PER_THREAD];
    uint64_t val[PACK_SLOTS_PER_THREAD];
    uint64_t ball[PACK_SLOTS_PER_THREAD];
    int64_t cnt = 0;
#pragma unroll
    for (int q = 0; q < PACK_SLOTS_PER_THREAD; ++q) {
      const int64_t s = s0 + (int64_t)q * PACK_BLOCK + threadIdx.x;
      bool keep = false;
      code[q] = 0;
      val[q] = 0;
      if (s < T.slots) {
        if (T.direct) {
          code[q] = s;
          val[q] = T.table[s];
          keep = true;
        } else {
          const uint64_t key = T.table[2 * s];
          code[q] = (int64_t)key - 1;
          val[q] = T.table[2 * s + 1];
          keep = key != 0;
        }
        // a zero sum is dropped (for fp64 both signed zeros)
        keep = keep && (T.f64 ? (val[q] << 1) != 0 : val[q] != 0);
      }
      ball[q] = __ballot(keep);
      cnt += __popcll(ball[q]);
    }
    if (lane == 0) s_wave[wave] = cnt;
    __syncthreads();
    int64_t tot = 0, pos = 0;
    for (int w = 0; w < PACK_BLOCK / 64; ++w) {
      if (w == wave) pos = tot;
      tot += s_wave[w];
    }
    if (threadIdx.x == 0)
      s_base = tot ? (int64_t)atomicAdd(T.count, (unsigned long long)tot) : 0;
    __syncthreads();
    const int64_t base = s_base;
    const uint64_t lt = (1ull << lane) - 1;
    const int nx = T.la.nx;
    int64_t* oc = static_cast<int64_t*>(T.out_c);
#pragma unroll
    for (int q = 0; q < PACK_SLOTS_PER_THREAD; ++q) {
      if (ball[q] & (1ull << lane)) {
        const int64_t at = base + pos + __popcll(ball[q] & lt);
        if (at < T.out_cap) {
          uint64_t c = (uint64_t)code[q];
          for (int v = 0; v < nx; ++v) T.out_x[at * nx + v] = decode_step_fast(T.la, v, c);
          oc[at] = (int64_t)val[q];
        }
      }
      pos += __popcll(ball[q]);
    }
    __syncthreads();   // s_wave and s_base are reused by the next unit
  }
}

// ------------------------------------------------------------ counts
// One workgroup: every task's count (or -(status) after a device error) as
// two tagged words in host-mapped memory.
__global__ void __launch_bounds__(PACK_BLOCK) k_pack_post(void* table) {
  const PackView P = view(table);
  const int nt = P.h->ntasks;
  const uint32_t err = P.h->err;
  const uint64_t tag = (uint64_t)(uint32_t)P.h->seq << 32;
  for (int k = threadIdx.x; k < nt; k += PACK_BLOCK) {
    int64_t n = (int64_t)*P.tasks[k].count;
    if (n > P.tasks[k].out_cap) n = -(int64_t)KP_E_CAPACITY;
    if (err) n = -(int64_t)first_error(err);
    const uint64_t w = (uint64_t)n;
    __hip_atomic_store(&P.h->post[2 * k], tag | (w & 0xffffffffu), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&P.h->post[2 * k + 1], tag | (w >> 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace

size_t pack_table_bytes(int max_tasks) {
  return sizeof(PackHeader) + 3 * sizeof(int64_t) * ((size_t)max_tasks + 1) +
         sizeof(PackTask) * (size_t)max_tasks;
}

hipError_t launch_pack_boxes(const int32_t* const* vals, const int64_t* n, const int32_t* nv,
                             int nseg, uint64_t* post_dev, uint64_t seq, hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_boxes, dim3((unsigned)nseg), dim3(PACK_BOX_BLOCK), 0, s, vals, n, nv,
                     post_dev, seq);
  return hipGetLastError();
}

hipError_t launch_pack_run(void* table_dev, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_prep, dim3((unsigned)grid), dim3(PACK_BLOCK), 0, s, table_dev);
  hipLaunchKernelGGL(k_pack_mul, dim3((unsigned)grid), dim3(PACK_BLOCK), 0, s, table_dev);
  hipLaunchKernelGGL(k_pack_compact, dim3((unsigned)grid), dim3(PACK_BLOCK), 0, s, table_dev);
  hipLaunchKernelGGL(k_pack_post, dim3(1), dim3(PACK_BLOCK), 0, s, table_dev);
  return hipGetLastError();
}

}  // namespace kp
