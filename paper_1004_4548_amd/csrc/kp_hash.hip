// kp_hash.hip -- hash-table accumulation for highly sparse products, and the
// Poisson split.
//
// Section 3.2 replaces the dense coefficient array with a hash table keyed by
// the product's code: a product whose code is already present adds its
// coefficient, otherwise it is inserted.  The paper's table is a bucketed,
// cache-blocked CPU design and mentions linear probing as an alternative; on
// gfx950 the table is one open-addressing array of 16-byte slots in HBM
// {code + 1, coefficient} (0 marks an empty slot), probed linearly from a
// multiplicative hash of the code.  A slot is claimed with a device-scope
// 64-bit compare-and-swap on the key and the coefficient is accumulated with a
// 64-bit atomic add (integer, or fp64 add), so concurrent insertions of the
// same code from any compute unit combine without locks.  Compaction reads
// the table once, selects non-empty slots with a nonzero coefficient by
// wavefront ballot and writes them contiguously.  Exact 128-bit sums of
// int64 products use 32-byte slots {code + 1, low word, high word, unused};
// the low word's atomic add returns its previous value, and the carry out of
// that add goes into the high word with the product's high word.
//
// Poisson series (Section 2, eq. werner with the factor 1/2): every pair
// contributes +-1/2 ca cb to the term of the difference and of the sum of the
// trigonometric arguments.  With the product's balanced trig code ky and the
// polynomial code kx in [0, Wx), the combined code K = kx + Wx * ky of a
// piece is kx_a + kx_b + Wx (ky_a +- ky_b); K < 0 exactly when ky < 0, and
// then the canonical form (first multiplier positive) is kx + Wx |ky|
// = 2 kx - K with the sign of a sine flipped.  A sine with ky = 0
// (0 <= K < Wx) is dropped.
#include <climits>
#include <type_traits>

#include "kp_internal.h"

namespace kp {

namespace {

constexpr int HASH_BLOCK = 256;
constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;   // 2^64 / golden ratio (Fibonacci hashing)

__device__ __forceinline__ void slot_add(uint64_t* c, int64_t v) {
  atomicAdd((unsigned long long*)c, (unsigned long long)v);
}
__device__ __forceinline__ void slot_add(uint64_t* c, double v) {
  unsafeAtomicAdd(reinterpret_cast<double*>(c), v);
}
__device__ __forceinline__ void slot_add(uint64_t* c, I128 v) {
  const uint64_t old = atomicAdd((unsigned long long*)c, (unsigned long long)v.lo);
  const uint64_t carry = old + v.lo < old ? 1u : 0u;
  atomicAdd((unsigned long long*)(c + 1), (unsigned long long)((uint64_t)v.hi + carry));
}

// 64-bit words per table slot: the key and one coefficient, padded to a
// power of two.
template <typename T>
constexpr int slot_words() {
  return sizeof(T) == 16 ? 4 : 2;
}

__device__ __forceinline__ uint64_t home_slot(int64_t code, uint64_t cap) {
  // multiplicative hash, then mapped onto [0, cap) by a high multiply
  return __umul64hi((uint64_t)code * GOLDEN, cap);
}

__device__ __forceinline__ uint64_t key_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Probe from slot s (whose key word read `cur`) until the key is found or
// claimed; at most max_probe slots are visited before the table is declared
// full.  An occupied slot is skipped after a plain (atomic) load; only an
// empty slot costs a compare-and-swap.
// Returns the number of slots visited beyond the home slot.
template <typename T>
__device__ __noinline__ int64_t table_probe(uint64_t* __restrict__ table, uint64_t cap,
                                            int64_t max_probe, uint64_t s, uint64_t cur,
                                            uint64_t key, T v, uint32_t* err) {
  for (int64_t p = 0; p < max_probe; ++p) {
    uint64_t* ks = table + slot_words<T>() * s;
    if (p > 0) cur = key_load(ks);
    if (cur == 0) {
      cur = atomicCAS((unsigned long long*)ks, 0ull, (unsigned long long)key);
      if (cur == 0) cur = key;
    }
    if (cur == key) {
      slot_add(ks + 1, v);
      return p;
    }
    s = s + 1 == cap ? 0 : s + 1;
  }
  atomicOr(err, ERR_CAPACITY);
  return max_probe;
}

// Adds a thread's counts into the context's statistics (one atomic per wavefront).
__device__ __forceinline__ void add_stats(unsigned long long* stats, int64_t ins, int64_t probes) {
  for (int off = 32; off > 0; off >>= 1) {
    ins += __shfl_xor(ins, off);
    probes += __shfl_xor(probes, off);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&stats[0], (unsigned long long)ins);
    atomicAdd(&stats[1], (unsigned long long)probes);
  }
}

// Insert-or-accumulate of NB independent contributions.  The key words of
// their home slots are read first, all NB loads in flight together; a slot
// holding the key gets the coefficient added atomically, an empty one is
// claimed by compare-and-swap (0 = empty, otherwise code + 1), anything
// else continues probing linearly.  Concurrent insertions of one code
// combine in any order because the coefficient word only ever receives
// atomic adds.
template <typename T, int NB>
__device__ __forceinline__ int64_t table_insert_n(uint64_t* __restrict__ table, uint64_t cap,
                                                  int64_t max_probe, const int64_t* code,
                                                  const T* v, const bool* on, uint32_t* err) {
  int64_t extra = 0;
  uint64_t s[NB], cur[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    s[u] = home_slot(code[u], cap);
    cur[u] = on[u] ? key_load(table + slot_words<T>() * s[u]) : 0;
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    if (!on[u]) continue;
    const uint64_t key = (uint64_t)code[u] + 1;
    if (cur[u] == key)
      slot_add(table + slot_words<T>() * s[u] + 1, v[u]);
    else
      extra += table_probe<T>(table, cap, max_probe, s[u], cur[u], key, v[u], err);
  }
  return extra;
}

template <typename T>
__device__ inline T mul_coef(T a, T b, uint32_t narrow);
template <>
__device__ inline int64_t mul_coef<int64_t>(int64_t a, int64_t b, uint32_t narrow) {
  if (narrow & 2u) {
    int32_t x = ((int32_t)a << 8) >> 8, y = ((int32_t)b << 8) >> 8;
    return (int64_t)x * (int64_t)y;
  }
  if (narrow & 1u) return (int64_t)(int32_t)a * (int64_t)(int32_t)b;
  return (int64_t)((uint64_t)a * (uint64_t)b);
}
template <>
__device__ inline double mul_coef<double>(double a, double b, uint32_t) {
  return a * b;
}

// Factor coefficients of a value type: 128-bit sums take int64 factors.
template <typename T>
using factor_t = typename std::conditional<std::is_same<T, I128>::value, int64_t, T>::type;

// Exact product of two int64 coefficients.
__device__ inline I128 mul_wide(int64_t a, int64_t b) {
  return I128((uint64_t)a * (uint64_t)b, __mul64hi(a, b));
}

// Thread = one term of B (in registers); loops over a slice of A's rows,
// whose code and coefficient are wavefront-uniform (scalar loads), four rows
// per round so that four insertions are in flight.
template <typename T>
__global__ void __launch_bounds__(HASH_BLOCK)
k_hash_laurent(uint64_t* __restrict__ table, uint64_t cap, int64_t max_probe, Meta* meta,
               const int64_t* __restrict__ ak, const factor_t<T>* __restrict__ ac, int64_t na,
               const int64_t* __restrict__ bk, const factor_t<T>* __restrict__ bc, int64_t nb,
               int rows,
               unsigned long long* stats, const int32_t* __restrict__ a_sa,
               const int32_t* __restrict__ b_tb) {
  constexpr int NB = 4;
  const int64_t j0 = (int64_t)blockIdx.x * HASH_BLOCK + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * rows;
  const int64_t i1 = min(i0 + rows, na);
  const uint32_t narrow = meta->narrow;
  const bool live = j0 < nb;
  const int64_t j = live ? j0 : nb - 1;   // idle lanes stay for the statistics reduction
  const int64_t bj = bk[j];
  const factor_t<T> cb = bc[j];
  const int32_t tb = b_tb ? b_tb[j] : INT_MIN;
  int64_t ins = 0, extra = 0;
  for (int64_t i = live ? i0 : i1; i < i1; i += NB) {
    int64_t code[NB];
    T v[NB];
    bool on[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const bool in = i + u < i1;
      const int64_t r = in ? i + u : i;
      if constexpr (std::is_same<T, I128>::value)
        v[u] = mul_wide(ac[r], cb);
      else
        v[u] = mul_coef<T>(ac[r], cb, narrow);
      code[u] = ak[r] + bj;
      on[u] = in && v[u] != T(0) && (!a_sa || tb <= a_sa[r]);
      ins += on[u];
    }
    extra += table_insert_n<T, NB>(table, cap, max_probe, code, v, on, &meta->err);
  }
  if (stats) add_stats(stats, ins, extra);
}

// Harmonic order of a factor's term, saturated to int32.
__device__ __forceinline__ int32_t term_order(const DevLayout& L, const HarmonicSpec& H,
                                              int64_t ky) {
  const int64_t o = harmonic_order(L, (uint64_t)(ky < 0 ? -ky : ky), H);
  return (int32_t)min(o, (int64_t)INT_MAX);
}

// A factor term's multipliers (balanced digits of its canonical code ky >= 0)
// as signed bytes, variable k in byte k.
__device__ __forceinline__ uint4 pack_multipliers(const DevLayout& L, int64_t ky) {
  uint32_t w[4] = {0, 0, 0, 0};
  uint64_t u = (uint64_t)(ky < 0 ? -ky : ky);
  for (int v = L.ny - 1; v >= 0; --v) {
    const int32_t d = decode_y_step(L, v, u);
    w[v >> 2] |= ((uint32_t)d & 0xFFu) << (8 * (v & 3));
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ void __launch_bounds__(HASH_BLOCK)
k_poisson_prep(int64_t Wx, const int64_t* __restrict__ ax, const int64_t* __restrict__ ay,
               const uint8_t* __restrict__ as, int64_t na, const int64_t* __restrict__ bx,
               const int64_t* __restrict__ by, const uint8_t* __restrict__ bs, int64_t nb,
               PoissonPrep P, DevLayout L, HarmonicSpec H, int harm_on) {
  const int64_t g = (int64_t)blockIdx.x * HASH_BLOCK + threadIdx.x;
  if (g < na) {
    P.ap[g] = ax[g] + Wx * ay[g];
    P.akx[g] = ax[g];
    P.at[g] = as[g];
    if (harm_on && P.ad) P.ad[g] = pack_multipliers(L, ay[g]);
    else if (harm_on) P.ao[g] = term_order(L, H, ay[g]);
  } else if (g < na + nb) {
    const int64_t j = g - na;
    P.bp[j] = bx[j] + Wx * by[j];
    P.bm[j] = bx[j] - Wx * by[j];
    P.bkx[j] = bx[j];
    P.bt[j] = bs[j];
    if (harm_on && P.bd) P.bd[j] = pack_multipliers(L, by[j]);
    else if (harm_on) P.bo[j] = term_order(L, H, by[j]);
  }
}

// The orders of a pair's difference and sum pieces, sum_k w_k |a_k -+ b_k|,
// from the factors' packed multipliers.
__device__ __forceinline__ void piece_orders(const uint4& a, const uint4& b, const RadixArgs& R,
                                             int64_t* om, int64_t* op) {
  int64_t m = 0, p = 0;
  const int ny = R.dec.ny;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t x = q == 0 ? a.x : q == 1 ? a.y : q == 2 ? a.z : a.w;
    const uint32_t y = q == 0 ? b.x : q == 1 ? b.y : q == 2 ? b.z : b.w;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * q + r;
      if (k < ny) {
        const int32_t da = (int32_t)(int8_t)(x >> (8 * r));
        const int32_t db = (int32_t)(int8_t)(y >> (8 * r));
        m += (int64_t)R.harm.w[k] * abs(da - db);
        p += (int64_t)R.harm.w[k] * abs(da + db);
      }
    }
  }
  *om = m;
  *op = p;
}

// A truncated pair makes no piece when its factors' orders differ by more
// than the limit: both pieces' orders are at least that difference.
__device__ __forceinline__ bool pair_over(const RadixArgs& R, int64_t i, int64_t j) {
  if (!R.harm_on || R.harm_exact) return false;
  const int64_t d = (int64_t)R.P.ao[i] - (int64_t)R.P.bo[j];
  return (d < 0 ? -d : d) > R.harm.max_order;
}

// Key and signed value of one piece; false when the piece vanishes.
__device__ __forceinline__ bool poisson_piece(int64_t Wx, int64_t K, int64_t kx, int t, double v,
                                              int64_t* key, double* val) {
  int64_t pos = K;
  if (K < 0) {                 // ky < 0: fold to |ky|, sin(-a) = -sin(a)
    pos = 2 * kx - K;
    if (t) v = -v;
  } else if (t && K < Wx) {    // sin of the zero multiplier vector vanishes
    return false;
  }
  *key = 2 * pos + t;
  *val = v;
  return true;
}

// Thread = one term of B; every pair yields the difference piece (sign -1 for
// cos*sin) and the sum piece (sign -1 for sin*sin), each 1/2 ca cb.  Two
// pairs per round: four insertions in flight.
__global__ void __launch_bounds__(HASH_BLOCK)
k_hash_poisson(uint64_t* __restrict__ table, uint64_t cap, int64_t max_probe, Meta* meta,
               int64_t Wx, const int64_t* __restrict__ ap, const int64_t* __restrict__ akx,
               const uint8_t* __restrict__ at, const double* __restrict__ ac, int64_t na,
               const int64_t* __restrict__ bp, const int64_t* __restrict__ bm,
               const int64_t* __restrict__ bkx, const uint8_t* __restrict__ bt,
               const double* __restrict__ bc, int64_t nb, int rows,
               unsigned long long* stats) {
  const int64_t j0 = (int64_t)blockIdx.x * HASH_BLOCK + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * rows;
  const int64_t i1 = min(i0 + rows, na);
  const bool live = j0 < nb;
  const int64_t j = live ? j0 : nb - 1;   // idle lanes stay for the statistics reduction
  int64_t ins = 0, extra = 0;
  const int64_t Bp = bp[j], Bm = bm[j], kxb = bkx[j];
  const int tb = bt[j];
  const double cb = bc[j];
  for (int64_t i = live ? i0 : i1; i < i1; i += 2) {
    int64_t code[4];
    double v[4];
    bool on[4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const bool in = i + u < i1;
      const int64_t r = in ? i + u : i;
      const int ta = at[r];
      const double h = 0.5 * (ac[r] * cb);
      const int64_t kx = akx[r] + kxb;
      const int t = ta ^ tb;
      const double sm = (!ta && tb) ? -h : h;   // cos a sin b: -1/2 sin(a - b)
      const double sp = (ta && tb) ? -h : h;    // sin a sin b: -1/2 cos(a + b)
      on[2 * u] = in && h != 0.0 && poisson_piece(Wx, ap[r] + Bm, kx, t, sm, &code[2 * u], &v[2 * u]);
      on[2 * u + 1] =
          in && h != 0.0 && poisson_piece(Wx, ap[r] + Bp, kx, t, sp, &code[2 * u + 1], &v[2 * u + 1]);
      if (!on[2 * u]) code[2 * u] = 0;
      if (!on[2 * u + 1]) code[2 * u + 1] = 0;
      ins += on[2 * u] + on[2 * u + 1];
    }
    extra += table_insert_n<double, 4>(table, cap, max_probe, code, v, on, &meta->err);
  }
  if (stats) add_stats(stats, ins, extra);
}

// ------------------------------------------------------------ compaction
constexpr int COMPACT_PER = 16;

template <typename T>
__global__ void __launch_bounds__(HASH_BLOCK)
k_hash_compact(const uint64_t* __restrict__ table, int64_t cap, Meta* meta,
               int64_t* __restrict__ out_k, T* __restrict__ out_c, int64_t out_cap) {
  __shared__ int64_t s_wave[HASH_BLOCK / 64];
  __shared__ int64_t s_base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t chunk = (int64_t)HASH_BLOCK * COMPACT_PER;
  for (int64_t base = (int64_t)blockIdx.x * chunk; base < cap; base += (int64_t)gridDim.x * chunk) {
    uint64_t key[COMPACT_PER];
    T val[COMPACT_PER];
    uint64_t ball[COMPACT_PER];
    int64_t wave_cnt = 0;
#pragma unroll
    for (int r = 0; r < COMPACT_PER; ++r) {
      const int64_t s = base + r * HASH_BLOCK + threadIdx.x;
      bool f = false;
      key[r] = 0;
      val[r] = T(0);
      if (s < cap) {
        const uint4* sl = reinterpret_cast<const uint4*>(table) + (slot_words<T>() / 2) * s;
        const uint4 w0 = sl[0];
        key[r] = ((uint64_t)w0.y << 32) | w0.x;
        uint64_t words[2] = {((uint64_t)w0.w << 32) | w0.z, 0};
        if constexpr (slot_words<T>() == 4) {
          const uint4 w1 = sl[1];
          words[1] = ((uint64_t)w1.y << 32) | w1.x;
        }
        __builtin_memcpy(&val[r], words, sizeof(T));
        f = key[r] != 0 && val[r] != T(0);
      }
      ball[r] = __ballot(f);
      wave_cnt += __popcll(ball[r]);
    }
    if (lane == 0) s_wave[wave] = wave_cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t tot = 0;
      for (int w = 0; w < HASH_BLOCK / 64; ++w) tot += s_wave[w];
      s_base = tot ? (int64_t)atomicAdd((unsigned long long*)&meta->out_count,
                                        (unsigned long long)tot)
                   : 0;
    }
    __syncthreads();
    int64_t pos = s_base;
    for (int w = 0; w < wave; ++w) pos += s_wave[w];
    const uint64_t lt = (1ull << lane) - 1;
#pragma unroll
    for (int r = 0; r < COMPACT_PER; ++r) {
      if (ball[r] & (1ull << lane)) {
        const int64_t p = pos + __popcll(ball[r] & lt);
        if (p < out_cap) {
          out_k[p] = (int64_t)(key[r] - 1);
          out_c[p] = val[r];
        }
      }
      pos += __popcll(ball[r]);
    }
    __syncthreads();
  }
}


// ------------------------------------------------------------ partitioned accumulation
// The same insert-or-accumulate with the table kept on chip.  Every nonzero
// product {code, value} is written once to HBM, grouped by the top bits of
// its multiplicative hash (level 1, with exact offsets from per-workgroup
// histograms, so the scatter needs no global atomics), then regrouped inside
// each level-1 partition by the next bits (level 2).  A level-2 bin holds
// about BIN_TARGET products, all of any one code; one workgroup accumulates
// a bin in an LDS open-addressing table and writes its nonzero terms.  HBM
// sees sequential runs instead of one random line per insertion.
constexpr int RADIX_BLOCK = RADIX_THREADS;   // count and scatter: threads over terms of B
constexpr int STAGE = 8192;          // entries staged per chunk (8 per thread): 128 KiB of LDS
constexpr int RADIX_MAX_L = 10;      // at most 1024 partitions per level
constexpr int SPLIT_BLOCK = 1024;
// A bin's LDS table has 2^LOG slots of 8 + 8 bytes (LOG 11, 12 or 13: 32, 64
// or 128 KiB, four, two or one workgroup per CU) and 2^LOG / 8 threads.
constexpr int BIN_PER_THREAD = 8;
constexpr int BIN_STACK = 72;   // code intervals of a bin's overflow passes (depth <= 64)

__device__ __forceinline__ uint64_t code_hash(int64_t code) { return (uint64_t)code * GOLDEN; }
__device__ __forceinline__ uint32_t part1(uint64_t h, int l1) { return (uint32_t)(h >> (64 - l1)); }
__device__ __forceinline__ uint32_t part2(uint64_t h, int l1, int l2) {
  return (uint32_t)(h >> (64 - l1 - l2)) & ((1u << l2) - 1);
}
template <int LOG>
__device__ __forceinline__ uint32_t bin_slot(uint64_t h, int l1, int l2) {
  return (uint32_t)(h >> (64 - l1 - l2 - LOG)) & ((1u << LOG) - 1);
}

// Every nonzero product of this thread: its term j of B against rows
// [i0, i1) of A.  KIND 0: Laurent int64, 1: Laurent fp64, 2: Poisson (two
// pieces per pair), 3: Laurent exact 128-bit sums, 4: Poisson cut by
// harmonic order.  f(code, value bits).
template <int KIND, typename F>
__device__ __forceinline__ void each_product(const RadixArgs& R, uint32_t narrow, F&& f) {
  const int64_t j = (int64_t)blockIdx.x * RADIX_BLOCK + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * R.rows;
  const int64_t i1 = min(i0 + R.rows, R.na);
  if (j >= R.nb) return;
  if constexpr (KIND == 2 || KIND == 4) {
    constexpr bool CUT = KIND == 4;
    const double* ac = static_cast<const double*>(R.ac);
    const int64_t Bp = R.P.bp[j], Bm = R.P.bm[j], kxb = R.P.bkx[j];
    const int tb = R.P.bt[j];
    const double cb = static_cast<const double*>(R.bc)[j];
    const uint4 bd = CUT && R.harm_exact ? R.P.bd[j] : uint4{};
    for (int64_t i = i0; i < i1; ++i) {
      if (CUT && pair_over(R, i, j)) continue;
      bool km = true, kp = true;   // the pieces within the order limit
      if (CUT && R.harm_exact) {
        int64_t om, op;
        piece_orders(R.P.ad[i], bd, R, &om, &op);
        km = om <= R.harm.max_order;
        kp = op <= R.harm.max_order;
        if (!km && !kp) continue;
      }
      const int ta = R.P.at[i];
      const double h = 0.5 * (ac[i] * cb);
      if (h == 0.0) continue;
      const int64_t kx = R.P.akx[i] + kxb;
      const int t = ta ^ tb;
      const double sm = (!ta && tb) ? -h : h;   // cos a sin b: -1/2 sin(a - b)
      const double sp = (ta && tb) ? -h : h;    // sin a sin b: -1/2 cos(a + b)
      int64_t key;
      double v;
      if (km && poisson_piece(R.Wx, R.P.ap[i] + Bm, kx, t, sm, &key, &v))
        f(key, __double_as_longlong(v));
      if (kp && poisson_piece(R.Wx, R.P.ap[i] + Bp, kx, t, sp, &key, &v))
        f(key, __double_as_longlong(v));
    }
  } else {
    using T = typename std::conditional<KIND == 1, double, int64_t>::type;
    const T* ac = static_cast<const T*>(R.ac);
    const int64_t bj = R.bk[j];
    const T cb = static_cast<const T*>(R.bc)[j];
    const int32_t tb = R.a_sa ? R.b_tb[j] : INT_MIN;
    for (int64_t i = i0; i < i1; ++i) {
      if (R.a_sa && tb > R.a_sa[i]) continue;   // over the degree limit
      if constexpr (KIND == 3) {   // exact sums: the pair's indices (the bins multiply)
        if (ac[i] == 0 || cb == 0) continue;
        f(R.ak[i] + bj, (int64_t)(((uint64_t)i << 32) | (uint64_t)j));
      } else {
        const T v = mul_coef<T>(ac[i], cb, narrow);
        if (v == T(0)) continue;
        int64_t bits;
        __builtin_memcpy(&bits, &v, 8);
        f(R.ak[i] + bj, bits);
      }
    }
  }
}

// Rows [r0, r0 + CR) of A against this thread's term j of B (CR = 8 for
// Laurent, 4 for Poisson, whose pairs give two pieces): up to 8 products in
// fixed slots, valid where `mask` has the slot's bit.
template <int KIND>
__device__ __forceinline__ uint32_t chunk_products(const RadixArgs& R, uint32_t narrow, int64_t j,
                                                   int64_t r0, int64_t r1, int64_t (&code)[8],
                                                   int64_t (&bits)[8]) {
  uint32_t mask = 0;
  if (j >= R.nb) return 0;
  if constexpr (KIND == 2 || KIND == 4) {
    constexpr bool CUT = KIND == 4;
    const double* ac = static_cast<const double*>(R.ac);
    const int64_t Bp = R.P.bp[j], Bm = R.P.bm[j], kxb = R.P.bkx[j];
    const int tb = R.P.bt[j];
    const double cb = static_cast<const double*>(R.bc)[j];
    // rows of A loaded two at a time (as for Laurent products below)
    int at[2];
    double ca[2];
    int64_t akx[2], ap[2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if ((u & 1) == 0) {
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          const int64_t i = min(r0 + u + w, r1 - 1);
          at[w] = R.P.at[i];
          ca[w] = ac[i];
          akx[w] = R.P.akx[i];
          ap[w] = R.P.ap[i];
        }
      }
      if (r0 + u >= r1) break;
      if (CUT && pair_over(R, r0 + u, j)) continue;
      bool km = true, kp = true;   // the pieces within the order limit
      if (CUT && R.harm_exact) {
        int64_t om, op;
        piece_orders(R.P.ad[r0 + u], R.P.bd[j], R, &om, &op);
        km = om <= R.harm.max_order;
        kp = op <= R.harm.max_order;
        if (!km && !kp) continue;
      }
      const int ta = at[u & 1];
      const double h = 0.5 * (ca[u & 1] * cb);
      if (h == 0.0) continue;
      const int64_t kx = akx[u & 1] + kxb;
      const int t = ta ^ tb;
      const double sm = (!ta && tb) ? -h : h;
      const double sp = (ta && tb) ? -h : h;
      double v;
      if (km && poisson_piece(R.Wx, ap[u & 1] + Bm, kx, t, sm, &code[2 * u], &v)) {
        bits[2 * u] = __double_as_longlong(v);
        mask |= 1u << (2 * u);
      }
      if (kp && poisson_piece(R.Wx, ap[u & 1] + Bp, kx, t, sp, &code[2 * u + 1], &v)) {
        bits[2 * u + 1] = __double_as_longlong(v);
        mask |= 1u << (2 * u + 1);
      }
    }
  } else {
    using T = typename std::conditional<KIND == 1, double, int64_t>::type;
    const T* ac = static_cast<const T*>(R.ac);
    const int64_t bj = R.bk[j];
    const T cb = static_cast<const T*>(R.bc)[j];
    const int32_t tb = R.a_sa ? R.b_tb[j] : INT_MIN;
    // rows of A are loaded four at a time (one wait per four rows, not one
    // per row); rows past the end repeat the last row and are not used
#pragma unroll
    for (int h = 0; h < 8; h += 4) {
      if (r0 + h >= r1) break;
      int64_t ka[4];
      T ca[4];
      int32_t sa[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = min(r0 + h + u, r1 - 1);
        ka[u] = R.ak[i];
        ca[u] = ac[i];
        sa[u] = R.a_sa ? R.a_sa[i] : INT_MAX;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (r0 + h + u >= r1) break;
        if (tb > sa[u]) continue;   // over the degree limit
        if constexpr (KIND == 3) {   // exact sums: the pair's indices (the bins multiply)
          if (ca[u] == 0 || cb == 0) continue;
          bits[h + u] = (int64_t)(((uint64_t)(r0 + h + u) << 32) | (uint64_t)j);
        } else {
          const T v = mul_coef<T>(ca[u], cb, narrow);
          if (v == T(0)) continue;
          __builtin_memcpy(&bits[h + u], &v, 8);
        }
        code[h + u] = ka[u] + bj;
        mask |= 1u << (h + u);
      }
    }
  }
  return mask;
}

// Exclusive scan of one value per thread over a workgroup of NT threads.
template <int NT>
__device__ __forceinline__ uint32_t block_scan1(uint32_t v, uint32_t* s_ws, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) s_ws[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < NT / 64; ++w) {
      const uint32_t x = s_ws[w];
      s_ws[w] = run;
      run += x;
    }
    s_ws[NT / 64] = run;
  }
  __syncthreads();
  const uint32_t r = s_ws[wave] + incl - v;
  *total = s_ws[NT / 64];
  __syncthreads();
  return r;
}

template <int KIND>
__global__ void __launch_bounds__(RADIX_BLOCK) k_radix_count(RadixArgs R) {
  __shared__ uint32_t hist[1 << RADIX_MAX_L];
  const int P1 = 1 << R.l1;
  for (int p = threadIdx.x; p < P1; p += RADIX_BLOCK) hist[p] = 0;
  __syncthreads();
  const uint32_t narrow = KIND == 0 ? R.meta->narrow : 0u;
  each_product<KIND>(R, narrow, [&](int64_t code, int64_t) {
    atomicAdd(&hist[part1(code_hash(code), R.l1)], 1u);
  });
  __syncthreads();
  const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  for (int p = threadIdx.x; p < P1; p += RADIX_BLOCK)
    R.counts[(int64_t)p * R.nblocks + blk] = hist[p];
}

// Exclusive scan of n values by one workgroup of BS threads, each taking a
// contiguous run; returns the total.  In place, 32-bit in-partition offsets
// (a partition of 2^32 products or more is reported as ERR_CAPACITY).
template <int BS, typename V>
__device__ int64_t block_scan_runs(V* a, int64_t n, Meta* meta) {
  __shared__ int64_t s_part[BS / 64];
  __shared__ int64_t s_total;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t per = (n + BS - 1) / BS;
  const int64_t r0 = min(n, (int64_t)tid * per), r1 = min(n, r0 + per);
  int64_t local = 0;
  for (int64_t r = r0; r < r1; ++r) local += (int64_t)a[r];
  int64_t incl = local;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) s_part[wave] = incl;
  __syncthreads();
  if (tid == 0) {
    int64_t run = 0;
    for (int w = 0; w < BS / 64; ++w) {
      const int64_t x = s_part[w];
      s_part[w] = run;
      run += x;
    }
    s_total = run;
  }
  __syncthreads();
  int64_t run = s_part[wave] + incl - local;
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t x = (int64_t)a[r];
    if (run > (int64_t)UINT32_MAX && sizeof(V) == 4) atomicOr(&meta->err, ERR_CAPACITY);
    a[r] = (V)run;
    run += x;
  }
  const int64_t total = s_total;
  __syncthreads();
  return total;
}

// One workgroup per level-1 partition: workgroup counts -> offsets within the
// partition, and the partition's total.
__global__ void __launch_bounds__(256) k_radix_scan_parts(RadixArgs R) {
  const int64_t p = blockIdx.x;
  const int64_t total = block_scan_runs<256>(R.counts + p * R.nblocks, R.nblocks, R.meta);
  if (threadIdx.x == 0) R.pstart[p] = total;
}

// Partition totals -> partition starts (pstart[P1] = number of products).
// Partition starts, and the level-2 bits for the products actually made:
// bins of at most half a table on average, as planned for all pairs, so that
// a truncated product (or one with many zero products) does not pay for
// bins it leaves empty.
__global__ void __launch_bounds__(1024) k_radix_scan_totals(RadixArgs R) {
  const int64_t P1 = (int64_t)1 << R.l1;
  const int64_t total = block_scan_runs<1024>(R.pstart, P1, R.meta);
  if (threadIdx.x == 0) {
    R.pstart[P1] = total;
    const int64_t half = ((int64_t)1 << R.bin_log) / 2;
    int bits = 1;
    while (bits < R.l1 + R.l2 && (half << bits) < total) ++bits;
    R.meta->radix_l2 = (uint32_t)max(0, bits - R.l1);
  }
}

// Products in chunks of 8 rows per thread: each chunk is counting-sorted by
// partition through LDS and written as contiguous runs (about 8 entries, one
// 128-byte line, per partition and chunk) after this workgroup's earlier
// runs in each partition.
template <int KIND>
__global__ void __launch_bounds__(RADIX_BLOCK) k_radix_scatter(RadixArgs R) {
  __shared__ uint4 stage[STAGE];
  __shared__ int64_t base[1 << RADIX_MAX_L];
  __shared__ uint32_t coff[1 << RADIX_MAX_L];
  __shared__ uint32_t done[1 << RADIX_MAX_L];
  __shared__ uint32_t s_ws[RADIX_BLOCK / 64 + 1];
  constexpr int CR = KIND == 2 || KIND == 4 ? 4 : 8;
  const int tid = threadIdx.x;
  const int P1 = 1 << R.l1;
  const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (tid < P1) {
    base[tid] = R.pstart[tid] + (int64_t)R.counts[(int64_t)tid * R.nblocks + blk];
    coff[tid] = 0;
    done[tid] = 0;
  }
  __syncthreads();
  const uint32_t narrow = KIND == 0 ? R.meta->narrow : 0u;
  const int l2 = (int)R.meta->radix_l2;
  const int64_t j = (int64_t)blockIdx.x * RADIX_BLOCK + tid;
  const int64_t i0 = (int64_t)blockIdx.y * R.rows;
  const int64_t i1 = min(i0 + R.rows, R.na);
  for (int64_t r0 = i0; r0 < i1; r0 += CR) {
    int64_t code[8], bits[8];
    const uint32_t mask = chunk_products<KIND>(R, narrow, j, r0, i1, code, bits);
    uint32_t part[8], rank[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if ((mask >> u) & 1u) {
        part[u] = part1(code_hash(code[u]), R.l1);
        rank[u] = atomicAdd(&coff[part[u]], 1u);
      }
    __syncthreads();
    const uint32_t mine = tid < P1 ? coff[tid] : 0u;
    uint32_t total;
    const uint32_t off = block_scan1<RADIX_BLOCK>(mine, s_ws, &total);
    if (tid < P1) coff[tid] = off;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if ((mask >> u) & 1u)
        stage[coff[part[u]] + rank[u]] = make_uint4((uint32_t)code[u],
                                                    (uint32_t)((uint64_t)code[u] >> 32),
                                                    (uint32_t)bits[u],
                                                    (uint32_t)((uint64_t)bits[u] >> 32));
    __syncthreads();
    for (uint32_t t = tid; t < total; t += RADIX_BLOCK) {
      const uint4 en = stage[t];
      const uint64_t h = code_hash((int64_t)(((uint64_t)en.y << 32) | en.x));
      const uint32_t p = part1(h, R.l1);
      const int64_t at = base[p] + done[p] + (t - coff[p]);
      R.ent1[at] = en;
      R.bin1[at] = (uint16_t)part2(h, R.l1, l2);   // for the split's histogram
    }
    __syncthreads();
    if (tid < P1) {
      done[tid] += mine;
      coff[tid] = 0;
    }
    __syncthreads();
  }
}

// One workgroup per level-1 partition: histogram by the level-2 bits, bin
// starts, and the regrouped copy, staged in chunks of STAGE entries like the
// scatter so that each bin receives contiguous runs.
__global__ void __launch_bounds__(SPLIT_BLOCK) k_radix_split(RadixArgs R) {
  static_assert(SPLIT_BLOCK * 8 == STAGE, "eight entries per thread and chunk");
  __shared__ uint4 stage[STAGE];
  __shared__ uint32_t h2[1 << RADIX_MAX_L];
  __shared__ uint32_t coff[1 << RADIX_MAX_L];
  __shared__ uint32_t done[1 << RADIX_MAX_L];
  __shared__ uint32_t s_ws[SPLIT_BLOCK / 64 + 1];
  const int tid = threadIdx.x;
  const int l2 = (int)R.meta->radix_l2;
  const int P2 = 1 << l2;
  const int64_t p = blockIdx.x;
  const int64_t s = R.pstart[p], e = R.pstart[p + 1];
  if (tid < P2) {
    h2[tid] = 0;
    coff[tid] = 0;
    done[tid] = 0;
  }
  __syncthreads();
  constexpr int U = 8;   // loads in flight per thread
  // Histogram from the 2-byte bin ids the scatter wrote beside the entries.
  // (Indices past the partition repeat its last entry, unused: loads without
  // a branch each, so that they are all in flight together.)
  constexpr int UB = 16;
  for (int64_t k0 = s + tid; k0 < e; k0 += (int64_t)SPLIT_BLOCK * UB) {
    uint32_t c[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) c[u] = R.bin1[min(k0 + (int64_t)u * SPLIT_BLOCK, e - 1)];
#pragma unroll
    for (int u = 0; u < UB; ++u)
      if (k0 + (int64_t)u * SPLIT_BLOCK < e) atomicAdd(&h2[c[u]], 1u);
  }
  __syncthreads();
  uint32_t all;
  const uint32_t boff = block_scan1<SPLIT_BLOCK>(tid < P2 ? h2[tid] : 0u, s_ws, &all);
  if (tid < P2) {
    h2[tid] = boff;
    R.bstart[p * P2 + tid] = s + boff;
  }
  if (p == ((int64_t)1 << R.l1) - 1 && tid == 0) R.bstart[(p + 1) * P2] = e;
  __syncthreads();
  // each chunk's entries are loaded while the previous chunk is written out
  uint4 en[U];
  const auto load_chunk = [&](int64_t c0) {
#pragma unroll
    for (int u = 0; u < U; ++u) en[u] = R.ent1[min(c0 + (int64_t)u * SPLIT_BLOCK + tid, e - 1)];
  };
  if (s < e) load_chunk(s);
  for (int64_t c0 = s; c0 < e; c0 += STAGE) {
    uint32_t bin[U], rank[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (c0 + (int64_t)u * SPLIT_BLOCK + tid < e) {
        const int64_t code = (int64_t)(((uint64_t)en[u].y << 32) | en[u].x);
        bin[u] = part2(code_hash(code), R.l1, l2);
        rank[u] = atomicAdd(&coff[bin[u]], 1u);
      }
    __syncthreads();
    const uint32_t mine = tid < P2 ? coff[tid] : 0u;
    uint32_t total;
    const uint32_t off = block_scan1<SPLIT_BLOCK>(mine, s_ws, &total);
    if (tid < P2) coff[tid] = off;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (c0 + (int64_t)u * SPLIT_BLOCK + tid < e) stage[coff[bin[u]] + rank[u]] = en[u];
    if (c0 + STAGE < e) load_chunk(c0 + STAGE);
    __syncthreads();
    for (uint32_t t = tid; t < total; t += SPLIT_BLOCK) {
      const uint4 x = stage[t];
      const uint32_t b = part2(code_hash((int64_t)(((uint64_t)x.y << 32) | x.x)), R.l1, l2);
      R.ent2[s + h2[b] + done[b] + (t - coff[b])] = x;
    }
    __syncthreads();
    if (tid < P2) {
      done[tid] += mine;
      coff[tid] = 0;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void lds_slot_add(int64_t* p, int64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}
__device__ __forceinline__ void lds_slot_add(double* p, double v) { atomicAdd(p, v); }
// 128-bit: the low word's returning add gives its carry, which the high word
// receives with the product's high word (each carry counted by the add that
// made it, so the sum is exact in any order)
__device__ __forceinline__ void lds_slot_add(I128* p, I128 v) {
  unsigned long long* w = reinterpret_cast<unsigned long long*>(p);
  const uint64_t old = atomicAdd(w, (unsigned long long)v.lo);
  const uint64_t carry = old + v.lo < old ? 1u : 0u;
  atomicAdd(w + 1, (unsigned long long)((uint64_t)v.hi + carry));
}

// One workgroup per level-2 bin: accumulate in an LDS table, then write the
// nonzero terms at an offset taken from the call's output counter.  A bin
// whose distinct codes overflow the table is redone by code interval.
template <typename T, int LOG>
__global__ void __launch_bounds__((1 << LOG) / BIN_PER_THREAD) k_radix_bins(RadixArgs R) {
  constexpr int BIN_SLOTS = 1 << LOG, BIN_BLOCK = BIN_SLOTS / BIN_PER_THREAD;
  __shared__ unsigned long long keys[BIN_SLOTS];
  __shared__ uint64_t vals_words[BIN_SLOTS * (sizeof(T) / 8)];   // (T may have a constructor)
  T* vals = reinterpret_cast<T*>(vals_words);
  __shared__ int64_t s_wave[BIN_BLOCK / 64];
  __shared__ int64_t s_base;
  __shared__ int s_over, s_sp;
  __shared__ unsigned long long s_lo[BIN_STACK], s_hi[BIN_STACK];
  // the grid covers the planned bins; the bins used are those of the level-2
  // bits chosen for the products actually made
  const int l2 = (int)R.meta->radix_l2;
  const int64_t b = blockIdx.x;
  if (b >= ((int64_t)1 << (R.l1 + l2))) return;
  const int64_t s = R.bstart[b], e = R.bstart[b + 1];
  if (s == e) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // The bin's first BIN_PER_THREAD entries per thread (a table's worth) are
  // loaded at once, before the table is cleared: one memory round trip for
  // the whole bin instead of one per entry.
  // (indices past the bin repeat its last entry, unused: loads without a
  // branch each, so that they are all in flight together)
  uint4 en[BIN_PER_THREAD];
#pragma unroll
  for (int u = 0; u < BIN_PER_THREAD; ++u)
    en[u] = R.ent2[min(s + tid + (int64_t)u * BIN_BLOCK, e - 1)];
  for (int i = tid; i < BIN_SLOTS; i += BIN_BLOCK) {
    keys[i] = 0;
    vals[i] = T(0);
  }
  if (tid == 0) s_over = 0;
  __syncthreads();
  int64_t ins = 0, extra = 0;
  const bool stats = R.stats != nullptr;
  // inserts the entry when its code lies in [ilo, ihi]; a full table sets
  // s_over (the bin is then redone in parts)
  const auto insert = [&](const uint4& x, uint64_t ilo, uint64_t ihi) {
    const int64_t code = (int64_t)(((uint64_t)x.y << 32) | x.x);
    if ((uint64_t)code < ilo || (uint64_t)code > ihi) return;
    T v;
    if constexpr (std::is_same<T, I128>::value) {   // exact: the entry holds the pair (i, j)
      v = mul_wide(static_cast<const int64_t*>(R.ac)[x.w], static_cast<const int64_t*>(R.bc)[x.z]);
    } else {
      const uint64_t bits = ((uint64_t)x.w << 32) | x.z;
      __builtin_memcpy(&v, &bits, 8);
    }
    const unsigned long long key = (unsigned long long)code + 1;
    uint32_t slot = bin_slot<LOG>(code_hash(code), R.l1, l2);
    // one compare-and-swap claims an empty slot or returns its key; the
    // probe loop has one exit test and the value is added after it
    unsigned long long c = atomicCAS(&keys[slot], 0ull, key);
    int q = 0;
#pragma nounroll
    while (c != 0 && c != key && q < BIN_SLOTS - 1) {
      ++q;
      slot = (slot + 1) & (BIN_SLOTS - 1);
      c = atomicCAS(&keys[slot], 0ull, key);
    }
    if (c != 0 && c != key) {   // every slot holds another code
      s_over = 1;
      return;
    }
    lds_slot_add(&vals[slot], v);
    if (stats) {
      ++ins;
      extra += q;
    }
  };
  T* out_c = static_cast<T*>(R.out_c);
  const int nx = R.dec.nx;
  const bool pairs = (nx & 1) == 0 && ((uintptr_t)R.out_x & 7) == 0;
  // Compacts the table to its front (thread tid owns slots tid + r *
  // BIN_BLOCK; every slot is read before any is rewritten), writes the
  // nonzero terms one per thread with all lanes busy at an offset taken from
  // the call's output counter, and clears the table when asked (another code
  // interval of the bin follows).
  const auto emit = [&](bool clear) {
    constexpr int PER = BIN_PER_THREAD;
    unsigned long long kk[PER];
    T vv[PER];
    uint64_t ball[PER];
    int64_t cnt = 0;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int i = r * BIN_BLOCK + tid;
      kk[r] = keys[i];
      vv[r] = vals[i];
      bool keep = kk[r] != 0 && vv[r] != T(0);
      // a truncated Poisson product drops the terms over the order limit
      // (key: 2 (kx + Wx |ky|) + is_sin)
      if (R.harm_on && !R.harm_exact && keep)
        keep = harmonic_order(R.dec, fdiv((uint64_t)(kk[r] - 1) >> 1, R.dec.dWx), R.harm) <=
               R.harm.max_order;
      ball[r] = __ballot(keep);
      cnt += __popcll(ball[r]);
    }
    if (lane == 0) s_wave[wave] = cnt;
    __syncthreads();
    int64_t tot = 0, pos = 0;
    for (int w = 0; w < BIN_BLOCK / 64; ++w) {
      if (w == wave) pos = tot;
      tot += s_wave[w];
    }
    if (tid == 0)
      s_base = tot ? (int64_t)atomicAdd((unsigned long long*)&R.meta->out_count,
                                        (unsigned long long)tot)
                   : 0;
    const uint64_t lt = (1ull << lane) - 1;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      if (ball[r] & (1ull << lane)) {
        const int64_t q = pos + __popcll(ball[r] & lt);
        keys[q] = kk[r];
        vals[q] = vv[r];
      }
      pos += __popcll(ball[r]);
    }
    __syncthreads();
    const int64_t base = s_base;
    const int64_t n = min(tot, R.out_cap - base);
    for (int64_t t = tid; t < n; t += BIN_BLOCK) {
      const int64_t q = base + t;
      const uint64_t code = (uint64_t)(keys[t] - 1);
      if (R.out_t) {   // Poisson key: sin flag, then kx + Wx |ky|, decoded
        uint64_t c = code >> 1;
        R.out_t[q] = (uint8_t)(code & 1);
        uint64_t u = fdiv(c, R.dec.dWx);
        uint64_t kx = c - u * (uint64_t)R.dec.Wx;
        for (int v = 0; v < nx; ++v) R.out_x[q * nx + v] = decode_step_fast(R.dec, v, kx);
        const int ny = R.dec.ny;
        for (int v = ny - 1; v >= 0; --v) R.out_y[q * ny + v] = decode_y_step(R.dec, v, u);
      } else if (R.out_x) {   // decoded exponents, written as they are found
        uint64_t c = code;
        if (pairs) {
          int2* o = reinterpret_cast<int2*>(R.out_x + q * nx);
          for (int v = 0; v < nx; v += 2) {
            const int32_t lo = decode_step_fast(R.dec, v, c);
            o[v >> 1] = make_int2(lo, decode_step_fast(R.dec, v + 1, c));
          }
        } else {
          for (int v = 0; v < nx; ++v) R.out_x[q * nx + v] = decode_step_fast(R.dec, v, c);
        }
      } else {
        R.out_k[q] = (int64_t)code;
      }
      out_c[q] = vals[t];
    }
    if (clear) {
      __syncthreads();
      for (int i = tid; i < BIN_SLOTS; i += BIN_BLOCK) {
        keys[i] = 0;
        vals[i] = T(0);
      }
      __syncthreads();
    }
  };
#pragma unroll
  for (int u = 0; u < BIN_PER_THREAD; ++u)
    if (s + tid + (int64_t)u * BIN_BLOCK < e) insert(en[u], 0, ~0ull);
  // bins of many products per code can hold more entries than slots
  for (int64_t k = s + tid + (int64_t)BIN_PER_THREAD * BIN_BLOCK; k < e; k += BIN_BLOCK)
    insert(R.ent2[k], 0, ~0ull);
  __syncthreads();
  if (!s_over) {
    emit(false);
  } else {
    // More distinct codes than slots (the table is full; Section 3.2 resizes
    // and rehashes): the bin again, one code interval at a time, halving an
    // interval whose codes overflow the table.  An interval of at most
    // BIN_SLOTS codes always fits, so the halving ends.
    for (int i = tid; i < BIN_SLOTS; i += BIN_BLOCK) {
      keys[i] = 0;
      vals[i] = T(0);
    }
    if (tid == 0) {
      s_lo[0] = ~0ull;
      s_hi[0] = 0;
    }
    __syncthreads();
    uint64_t mn = ~0ull, mx = 0;
    for (int64_t k = s + tid; k < e; k += BIN_BLOCK) {
      const uint4 x = R.ent2[k];
      const uint64_t code = ((uint64_t)x.y << 32) | x.x;
      mn = code < mn ? code : mn;
      mx = code > mx ? code : mx;
    }
    atomicMin(&s_lo[0], (unsigned long long)mn);
    atomicMax(&s_hi[0], (unsigned long long)mx);
    if (tid == 0) s_sp = 1;
    __syncthreads();
    while (s_sp > 0) {
      const uint64_t ilo = s_lo[s_sp - 1], ihi = s_hi[s_sp - 1];
      __syncthreads();
      if (tid == 0) {
        s_over = 0;
        --s_sp;
      }
      __syncthreads();
      for (int64_t k = s + tid; k < e; k += BIN_BLOCK) insert(R.ent2[k], ilo, ihi);
      __syncthreads();
      if (s_over) {
        // the upper half is pushed first, so the lower half runs next
        if (tid == 0) {
          const uint64_t mid = ilo + (ihi - ilo) / 2;
          s_lo[s_sp] = mid + 1;
          s_hi[s_sp] = ihi;
          s_lo[s_sp + 1] = ilo;
          s_hi[s_sp + 1] = mid;
          s_sp += 2;
        }
        __syncthreads();
        for (int i = tid; i < BIN_SLOTS; i += BIN_BLOCK) {
          keys[i] = 0;
          vals[i] = T(0);
        }
        __syncthreads();
      } else {
        emit(true);
      }
    }
  }
  if (R.stats) add_stats(R.stats, ins, extra);
}

// ------------------------------------------------------------ bucketed table
// Section 3.2's table: N buckets of m slots in one array, a product of code
// e going to bucket e mod N, where it is added to the slot already holding e
// or appended after the bucket's last term; a full bucket sends it to an
// overflow area, which is searched whenever a full bucket is met.  On the
// GPU the bucket's slots are claimed in order by compare-and-swap (a
// concurrent append), so a code is in at most one slot of its bucket, and a
// code only reaches the overflow area when every slot of its bucket holds
// another code for good; the overflow area is an open-addressing table,
// since many insertions can overflow at a load the GPU table runs at, where
// the paper's list would be searched linearly.  A full overflow table is
// reported as a capacity error (the point at which the paper resizes).

__device__ __forceinline__ uint64_t mod_bucket(int64_t code, const BucketGeom& G) {
  const uint64_t c = (uint64_t)code;
  return c - fdiv(c, G.fN) * G.nbuckets;
}

// Slots visited beyond the first (m and the overflow table's probes for an
// overflowing product), with OVF_BIT set when the product went to the
// overflow table.
constexpr int64_t OVF_BIT = (int64_t)1 << 62;

template <typename T>
__device__ __forceinline__ int64_t bucket_probe(uint64_t* __restrict__ table, int m, uint64_t nbuckets,
                                             int64_t ovcap, int64_t max_probe, uint64_t base,
                                             uint64_t cur, uint64_t key, T v, uint32_t* err) {
  for (int k = 0; k < m; ++k) {
    uint64_t* ks = table + 2 * (base + (uint64_t)k);
    if (k > 0) cur = key_load(ks);
    if (cur == 0) {
      cur = atomicCAS((unsigned long long*)ks, 0ull, (unsigned long long)key);
      if (cur == 0) cur = key;
    }
    if (cur == key) {
      slot_add(ks + 1, v);
      return k;
    }
  }
  uint64_t* ov = table + 2 * nbuckets * (uint64_t)m;
  const uint64_t h = home_slot((int64_t)(key - 1), (uint64_t)ovcap);
  return OVF_BIT + m +
         table_probe<T>(ov, (uint64_t)ovcap, max_probe, h, key_load(ov + 2 * h), key, v, err);
}

// Thread = one term of B, rows of A wavefront-uniform, NB insertions with
// their first key loads in flight together (as the open-addressing kernel).
template <typename T>
__global__ void __launch_bounds__(HASH_BLOCK)
k_hash_laurent_bucket(uint64_t* __restrict__ table, BucketGeom G, int64_t max_probe, Meta* meta,
                      const int64_t* __restrict__ ak, const T* __restrict__ ac, int64_t na,
                      const int64_t* __restrict__ bk, const T* __restrict__ bc, int64_t nb,
                      int rows, unsigned long long* stats, const int32_t* __restrict__ a_sa,
                      const int32_t* __restrict__ b_tb) {
  constexpr int NB = 4;
  const int64_t j0 = (int64_t)blockIdx.x * HASH_BLOCK + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * rows;
  const int64_t i1 = min(i0 + rows, na);
  const uint32_t narrow = meta->narrow;
  const bool live = j0 < nb;
  const int64_t j = live ? j0 : nb - 1;   // idle lanes stay for the statistics reduction
  const int64_t bj = bk[j];
  const T cb = bc[j];
  const int32_t tb = b_tb ? b_tb[j] : INT_MIN;
  int64_t ins = 0, extra = 0, novf = 0;
  for (int64_t i = live ? i0 : i1; i < i1; i += NB) {
    uint64_t base[NB], cur[NB];
    int64_t code[NB];
    T v[NB];
    bool on[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const bool in = i + u < i1;
      const int64_t r = in ? i + u : i;
      v[u] = mul_coef<T>(ac[r], cb, narrow);
      code[u] = ak[r] + bj;
      on[u] = in && v[u] != T(0) && (!a_sa || tb <= a_sa[r]);
      ins += on[u];
      base[u] = mod_bucket(code[u], G) * (uint64_t)G.m;
      cur[u] = on[u] ? key_load(table + 2 * base[u]) : 0;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (!on[u]) continue;
      const uint64_t key = (uint64_t)code[u] + 1;
      if (cur[u] == key) {
        slot_add(table + 2 * base[u] + 1, v[u]);
      } else {
        const int64_t pr = bucket_probe<T>(table, G.m, G.nbuckets, G.ovcap, max_probe, base[u],
                                           cur[u], key, v[u], &meta->err);
        extra += pr & (OVF_BIT - 1);
        novf += pr >> 62;
      }
    }
  }
  if (stats) {
    add_stats(stats, ins, extra);
    for (int off = 32; off > 0; off >>= 1) novf += __shfl_xor(novf, off);
    if ((threadIdx.x & 63) == 0 && novf) atomicAdd(&stats[2], (unsigned long long)novf);
  }
}

// The paper's term order for the hashed product: each factor's terms by code
// mod N, so that consecutive products of a row go to consecutive buckets.
// One workgroup per factor: a counting sort on MOD_BINS bins of the residue
// (the order within a bin is unspecified), ranks kept in global scratch.
constexpr int MOD_BLOCK = 1024;
constexpr int MOD_BINS = 16384;

__global__ void __launch_bounds__(MOD_BLOCK) k_mod_order(ModOrder O, BucketGeom G) {
  __shared__ int32_t hist[MOD_BINS];
  __shared__ uint32_t s_ws[MOD_BLOCK / 64 + 1];
  const int f = blockIdx.x;
  const int64_t n = O.n[f];
  const int64_t* __restrict__ kin = O.k_in[f];
  // bin = floor(MOD_BINS * (code mod N) / N), exact in 64 bits for N < 2^40
  auto bin_of = [&](int64_t code) -> int {
    const uint64_t r = mod_bucket(code, G);
    return (int)fdiv(r * (uint64_t)MOD_BINS, G.fN);
  };
  for (int b = threadIdx.x; b < MOD_BINS; b += MOD_BLOCK) hist[b] = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += MOD_BLOCK)
    O.rank[f][i] = atomicAdd(&hist[bin_of(kin[i])], 1);
  __syncthreads();
  // exclusive scan of the bins: MOD_BINS / MOD_BLOCK consecutive bins per thread
  constexpr int PER = MOD_BINS / MOD_BLOCK;
  uint32_t part = 0;
  for (int q = 0; q < PER; ++q) part += (uint32_t)hist[threadIdx.x * PER + q];
  uint32_t total;
  uint32_t run = block_scan1<MOD_BLOCK>(part, s_ws, &total);
  for (int q = 0; q < PER; ++q) {
    const int b = threadIdx.x * PER + q;
    const uint32_t c = (uint32_t)hist[b];
    hist[b] = (int32_t)run;
    run += c;
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += MOD_BLOCK) {
    const int64_t code = kin[i];
    const int64_t pos = hist[bin_of(code)] + O.rank[f][i];
    O.k_out[f][pos] = code;
    O.c_out[f][pos] = O.c_in[f][i];
    if (O.t_in[f]) O.t_out[f][pos] = O.t_in[f][i];
  }
}

}  // namespace

hipError_t launch_hash_laurent(const HashBufs& H, kp_dtype dt, const int64_t* ak, const void* ac,
                               int64_t na, const int64_t* bk, const void* bc, int64_t nb,
                               int rows, hipStream_t s) {
  if (rows < 1) rows = 1;
  dim3 grid((unsigned)((nb + HASH_BLOCK - 1) / HASH_BLOCK), (unsigned)((na + rows - 1) / rows));
  if (H.ev0) (void)hipEventRecord(H.ev0, s);
  if (dt == KP_F64)
    hipLaunchKernelGGL(k_hash_laurent<double>, grid, dim3(HASH_BLOCK), 0, s, H.table,
                       (uint64_t)H.cap, H.max_probe, H.meta, ak, (const double*)ac, na, bk,
                       (const double*)bc, nb, rows, H.stats, H.a_sa, H.b_tb);
  else if (dt == KP_I128)
    hipLaunchKernelGGL(k_hash_laurent<I128>, grid, dim3(HASH_BLOCK), 0, s, H.table,
                       (uint64_t)H.cap, H.max_probe, H.meta, ak, (const int64_t*)ac, na, bk,
                       (const int64_t*)bc, nb, rows, H.stats, H.a_sa, H.b_tb);
  else
    hipLaunchKernelGGL(k_hash_laurent<int64_t>, grid, dim3(HASH_BLOCK), 0, s, H.table,
                       (uint64_t)H.cap, H.max_probe, H.meta, ak, (const int64_t*)ac, na, bk,
                       (const int64_t*)bc, nb, rows, H.stats, H.a_sa, H.b_tb);
  if (H.ev1) (void)hipEventRecord(H.ev1, s);
  return hipGetLastError();
}

hipError_t launch_poisson_prep(int64_t Wx, const int64_t* ax, const int64_t* ay, const uint8_t* as,
                               int64_t na, const int64_t* bx, const int64_t* by,
                               const uint8_t* bs, int64_t nb, const PoissonPrep& P, hipStream_t s,
                               const DevLayout* L, const HarmonicSpec* H) {
  const int64_t n = na + nb;
  if (n == 0) return hipSuccess;
  const int harm_on = L && H && ((P.ao && P.bo) || (P.ad && P.bd)) ? 1 : 0;
  hipLaunchKernelGGL(k_poisson_prep, dim3((unsigned)((n + HASH_BLOCK - 1) / HASH_BLOCK)),
                     dim3(HASH_BLOCK), 0, s, Wx, ax, ay, as, na, bx, by, bs, nb, P,
                     harm_on ? *L : DevLayout{}, harm_on ? *H : HarmonicSpec{}, harm_on);
  return hipGetLastError();
}

hipError_t launch_hash_poisson(const HashBufs& H, int64_t Wx, const PoissonPrep& P,
                               const double* ac, int64_t na, const double* bc, int64_t nb,
                               int rows, hipStream_t s) {
  if (rows < 1) rows = 1;
  dim3 grid((unsigned)((nb + HASH_BLOCK - 1) / HASH_BLOCK), (unsigned)((na + rows - 1) / rows));
  if (H.ev0) (void)hipEventRecord(H.ev0, s);
  hipLaunchKernelGGL(k_hash_poisson, grid, dim3(HASH_BLOCK), 0, s, H.table, (uint64_t)H.cap,
                     H.max_probe, H.meta, Wx, P.ap, P.akx, P.at, ac, na, P.bp, P.bm, P.bkx, P.bt,
                     bc, nb, rows, H.stats);
  if (H.ev1) (void)hipEventRecord(H.ev1, s);
  return hipGetLastError();
}

hipError_t launch_hash_compact(const HashBufs& H, kp_dtype dt, hipStream_t s) {
  const int64_t cap = H.cap;
  const int64_t chunk = (int64_t)HASH_BLOCK * COMPACT_PER;
  int64_t blocks = (cap + chunk - 1) / chunk;
  if (blocks > 8192) blocks = 8192;
  if (dt == KP_F64)
    hipLaunchKernelGGL(k_hash_compact<double>, dim3((unsigned)blocks), dim3(HASH_BLOCK), 0, s,
                       H.table, cap, H.meta, H.out_k, (double*)H.out_c, H.out_cap);
  else if (dt == KP_I128)
    hipLaunchKernelGGL(k_hash_compact<I128>, dim3((unsigned)blocks), dim3(HASH_BLOCK), 0, s,
                       H.table, cap, H.meta, H.out_k, (I128*)H.out_c, H.out_cap);
  else
    hipLaunchKernelGGL(k_hash_compact<int64_t>, dim3((unsigned)blocks), dim3(HASH_BLOCK), 0, s,
                       H.table, cap, H.meta, H.out_k, (int64_t*)H.out_c, H.out_cap);
  return hipGetLastError();
}

hipError_t launch_radix(const RadixArgs& R0, int kind, hipStream_t s) {
  RadixArgs R = R0;
  if (R.na == 0 || R.nb == 0) return hipSuccess;
  if (kind == 2 && R.harm_on) kind = 4;   // Poisson products cut by harmonic order
  const dim3 grid((unsigned)((R.nb + RADIX_BLOCK - 1) / RADIX_BLOCK),
                  (unsigned)((R.na + R.rows - 1) / R.rows));
  R.nblocks = (int64_t)grid.x * grid.y;
  const unsigned P1 = 1u << R.l1;
  if (R.ev0) (void)hipEventRecord(R.ev0, s);
  if (kind == 4)
    hipLaunchKernelGGL(k_radix_count<4>, grid, dim3(RADIX_BLOCK), 0, s, R);
  else if (kind == 3)
    hipLaunchKernelGGL(k_radix_count<3>, grid, dim3(RADIX_BLOCK), 0, s, R);
  else if (kind == 2)
    hipLaunchKernelGGL(k_radix_count<2>, grid, dim3(RADIX_BLOCK), 0, s, R);
  else if (kind == 1)
    hipLaunchKernelGGL(k_radix_count<1>, grid, dim3(RADIX_BLOCK), 0, s, R);
  else
    hipLaunchKernelGGL(k_radix_count<0>, grid, dim3(RADIX_BLOCK), 0, s, R);
  hipLaunchKernelGGL(k_radix_scan_parts, dim3(P1), dim3(256), 0, s, R);
  hipLaunchKernelGGL(k_radix_scan_totals, dim3(1), dim3(1024), 0, s, R);
  if (kind == 4)
    hipLaunchKernelGGL(k_radix_scatter<4>, grid, dim3(RADIX_BLOCK), 0, s, R);
  else if (kind == 3)
    hipLaunchKernelGGL(k_radix_scatter<3>, grid, dim3(RADIX_BLOCK), 0, s, R);
  else if (kind == 2)
    hipLaunchKernelGGL(k_radix_scatter<2>, grid, dim3(RADIX_BLOCK), 0, s, R);
  else if (kind == 1)
    hipLaunchKernelGGL(k_radix_scatter<1>, grid, dim3(RADIX_BLOCK), 0, s, R);
  else
    hipLaunchKernelGGL(k_radix_scatter<0>, grid, dim3(RADIX_BLOCK), 0, s, R);
  hipLaunchKernelGGL(k_radix_split, dim3(P1), dim3(SPLIT_BLOCK), 0, s, R);
  const dim3 bins(P1 << R.l2), block((1u << R.bin_log) / BIN_PER_THREAD);
  if (kind == 3) {   // 128-bit sums: 24-byte slots, tables of at most 4096 (the planner's cap)
    if (R.bin_log >= 12)
      hipLaunchKernelGGL((k_radix_bins<I128, 12>), bins, dim3(4096 / BIN_PER_THREAD), 0, s, R);
    else
      hipLaunchKernelGGL((k_radix_bins<I128, 11>), bins, dim3(2048 / BIN_PER_THREAD), 0, s, R);
  } else if (R.bin_log == 13) {
    if (kind == 0) hipLaunchKernelGGL((k_radix_bins<int64_t, 13>), bins, block, 0, s, R);
    else hipLaunchKernelGGL((k_radix_bins<double, 13>), bins, block, 0, s, R);
  } else if (R.bin_log == 12) {
    if (kind == 0) hipLaunchKernelGGL((k_radix_bins<int64_t, 12>), bins, block, 0, s, R);
    else hipLaunchKernelGGL((k_radix_bins<double, 12>), bins, block, 0, s, R);
  } else {
    if (kind == 0) hipLaunchKernelGGL((k_radix_bins<int64_t, 11>), bins, block, 0, s, R);
    else hipLaunchKernelGGL((k_radix_bins<double, 11>), bins, block, 0, s, R);
  }
  if (R.ev1) (void)hipEventRecord(R.ev1, s);
  return hipGetLastError();
}

hipError_t launch_hash_laurent_bucket(const HashBufs& H, const BucketGeom& G, kp_dtype dt,
                                      const int64_t* ak, const void* ac, int64_t na,
                                      const int64_t* bk, const void* bc, int64_t nb, int rows,
                                      hipStream_t s) {
  if (rows < 1) rows = 1;
  dim3 grid((unsigned)((nb + HASH_BLOCK - 1) / HASH_BLOCK), (unsigned)((na + rows - 1) / rows));
  if (H.ev0) (void)hipEventRecord(H.ev0, s);
  if (dt == KP_F64)
    hipLaunchKernelGGL(k_hash_laurent_bucket<double>, grid, dim3(HASH_BLOCK), 0, s, H.table, G,
                       H.max_probe, H.meta, ak, (const double*)ac, na, bk, (const double*)bc, nb,
                       rows, H.stats, H.a_sa, H.b_tb);
  else
    hipLaunchKernelGGL(k_hash_laurent_bucket<int64_t>, grid, dim3(HASH_BLOCK), 0, s, H.table, G,
                       H.max_probe, H.meta, ak, (const int64_t*)ac, na, bk, (const int64_t*)bc, nb,
                       rows, H.stats, H.a_sa, H.b_tb);
  if (H.ev1) (void)hipEventRecord(H.ev1, s);
  return hipGetLastError();
}

hipError_t launch_mod_order(const ModOrder& O, const BucketGeom& G, hipStream_t s) {
  if (O.n[0] + O.n[1] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mod_order, dim3(2), dim3(MOD_BLOCK), 0, s, O, G);
  return hipGetLastError();
}

}  // namespace kp
