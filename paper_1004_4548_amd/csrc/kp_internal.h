// kp_internal.h -- shared definitions of the HIP path (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/kp.h"

namespace kp {

// ------------------------------------------------------------------ errors
// Device-detected errors are latched as bits (1 << status) in a 32-bit word.
enum : uint32_t {
  ERR_RANGE = 1u << KP_E_RANGE,
  ERR_NONCANONICAL = 1u << KP_E_NONCANONICAL,
  ERR_CAPACITY = 1u << KP_E_CAPACITY,
};

__host__ __device__ inline int first_error(uint32_t bits) {
  if (bits & ERR_RANGE) return KP_E_RANGE;
  if (bits & ERR_NONCANONICAL) return KP_E_NONCANONICAL;
  if (bits & ERR_CAPACITY) return KP_E_CAPACITY;
  return bits ? KP_E_DEVICE : KP_OK;
}

// -------------------------------------------------- invariant-divisor division
// Unsigned division of a 64-bit n by a fixed d >= 1 with one high multiply
// (Granlund & Montgomery 1994, the round-up method for N-bit operands):
//   l = ceil(log2 d),  m = floor(2^64 (2^l - d) / d) + 1,
//   t = mulhi(m, n),   n / d = (t + ((n - t) >> min(l,1))) >> max(l-1,0).
struct FastDiv {
  uint64_t m;
  uint64_t d;
  uint32_t s1, s2;
};

inline FastDiv make_fastdiv(uint64_t d) {
  FastDiv f{};
  f.d = d ? d : 1;
  uint32_t l = 0;
  while (l < 64 && (1ull << l) < f.d) ++l;
  unsigned __int128 num = ((unsigned __int128)(((l == 64) ? 0 : (1ull << l)) - f.d)) << 64;
  f.m = (uint64_t)(num / f.d) + 1;
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 0 ? l - 1 : 0;
  return f;
}

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ __forceinline__ uint64_t fdiv(uint64_t n, const FastDiv& f) {
  uint64_t t = mulhi64(f.m, n);
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

// The same method for 32-bit operands (one 32-bit high multiply), for
// divisors below 2^32.
struct FastDiv32 {
  uint32_t m, d;
  uint32_t s1, s2;
};

inline FastDiv32 make_fastdiv32(uint64_t d64) {
  FastDiv32 f{};
  const uint64_t d = d64 ? d64 : 1;
  if (d > 0xffffffffull) return f;   // unused: quotients of 32-bit values are then 0
  f.d = (uint32_t)d;
  uint32_t l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  const uint64_t num = ((l == 32 ? (1ull << 32) : (1ull << l)) - d) << 32;
  f.m = (uint32_t)(num / d + 1);
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 0 ? l - 1 : 0;
  return f;
}

__host__ __device__ __forceinline__ uint32_t fdiv32(uint32_t n, const FastDiv32& f) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t t = __umulhi(f.m, n);
#else
  const uint32_t t = (uint32_t)(((uint64_t)f.m * n) >> 32);
#endif
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

// ------------------------------------------------------------ device layout
// What the kernels need of a kp_layout, for one factor (encode) or for the
// product (decode), passed by value as a kernel argument.
struct DevLayout {
  int32_t nx, ny;
  int64_t Wx, Hy, nkeys;
  int32_t fmin[KP_MAX_VARS], fmax[KP_MAX_VARS];  // factor box (encode)
  int32_t fh[KP_MAX_VARS];                       // factor trig half-width (encode)
  int64_t xc[KP_MAX_VARS];
  int64_t xmin[KP_MAX_VARS];                     // product box minimum (decode)
  int64_t yc[KP_MAX_VARS];
  int64_t yh[KP_MAX_VARS];
  FastDiv dx[KP_MAX_VARS];                       // divide by product width xw_k
  FastDiv dy[KP_MAX_VARS];                       // divide by 2 yh_k + 1
  FastDiv dWx;
  FastDiv32 dx32[KP_MAX_VARS];                   // the same widths, 32-bit operands
};

DevLayout make_dev_layout(const kp_layout& L, int which);

// Truncation by weighted degree: keep product terms with
// sum_v w[v] e[v] <= max_degree.
struct TruncSpec {
  int32_t w[KP_MAX_VARS];
  int64_t max_degree;
};
hipError_t launch_degrees(const DevLayout& LA, const DevLayout& LB, const TruncSpec& T, int64_t na,
                          int64_t nb, const int64_t* ak, const int64_t* bk, int32_t* sa,
                          int32_t* tb, uint32_t* err, hipStream_t s);

// Per-term code map.  Returns an error bit (0 when fine).
__host__ __device__ inline uint32_t encode_term(const DevLayout& L, const int32_t* e,
                                                const int32_t* j, int is_sin, int64_t* kx,
                                                int64_t* ky) {
  uint32_t err = 0;
  int64_t x = 0;
  for (int v = 0; v < L.nx; ++v) {
    int32_t ev = e[v];
    if (ev < L.fmin[v] || ev > L.fmax[v]) err |= ERR_RANGE;
    x += L.xc[v] * (int64_t)(ev - L.fmin[v]);
  }
  *kx = x;
  if (L.ny > 0) {
    int64_t y = 0;
    for (int v = 0; v < L.ny; ++v) {
      int32_t jv = j[v];
      if (jv < -L.fh[v] || jv > L.fh[v]) err |= ERR_RANGE;
      y += L.yc[v] * (int64_t)jv;
    }
    // canonical: first nonzero multiplier positive (<=> y > 0), no sin(0)
    if (y < 0 || (y == 0 && is_sin)) err |= ERR_NONCANONICAL;
    *ky = y;
  }
  return err;
}

// Laurent product code -> exponents.
// Exponent v of the code whose quotient by the widths of variables < v is q;
// q becomes the quotient by the widths up to v.
__host__ __device__ __forceinline__ int32_t decode_step(const DevLayout& L, int v, uint64_t& q) {
  const uint64_t qq = fdiv(q, L.dx[v]);
  const int32_t e = (int32_t)((int64_t)(q - qq * L.dx[v].d) + L.xmin[v]);
  q = qq;
  return e;
}

// decode_step with a 32-bit division once the quotient fits in 32 bits
// (widths below 2^32).
__host__ __device__ __forceinline__ int32_t decode_step_fast(const DevLayout& L, int v, uint64_t& q) {
  if ((q >> 32) == 0 && L.dx32[v].d != 0) {
    const uint32_t q32 = (uint32_t)q;
    const uint32_t qq = fdiv32(q32, L.dx32[v]);
    const int32_t e = (int32_t)((int64_t)(q32 - qq * L.dx32[v].d) + L.xmin[v]);
    q = qq;
    return e;
  }
  return decode_step(L, v, q);
}

__host__ __device__ inline void decode_x(const DevLayout& L, uint64_t q, int32_t* e) {
  for (int v = 0; v < L.nx; ++v) e[v] = decode_step(L, v, q);
}

// Balanced digit v of |ky| (digits are found from v = ny - 1 down, y_0 most
// significant); u becomes the quotient for the next digit.
__host__ __device__ inline int32_t decode_y_step(const DevLayout& L, int v, uint64_t& u) {
  const uint64_t w = L.dy[v].d;
  const uint64_t h = (uint64_t)L.yh[v];
  const uint64_t s = u + h;
  const uint64_t qq = fdiv(s, L.dy[v]);
  const int64_t d = (int64_t)(s - qq * w) - (int64_t)h;
  u = qq;  // (u - d) / w == floor((u + h) / w)
  return (int32_t)d;
}

// |ky| -> canonical balanced digits, y_0 most significant.
__host__ __device__ inline void decode_y(const DevLayout& L, uint64_t u, int32_t* j) {
  for (int v = L.ny - 1; v >= 0; --v) j[v] = decode_y_step(L, v, u);
}

// Truncation of Poisson products by weighted harmonic order
// sum_k w_k |j_k| <= max_order (weights >= 0).
struct HarmonicSpec {
  int32_t w[KP_MAX_VARS];
  int64_t max_order;
};
// Order of the trigonometric part whose code is +-u (u = |ky|), saturated
// to int32 range.
__host__ __device__ inline int64_t harmonic_order(const DevLayout& L, uint64_t u,
                                                  const HarmonicSpec& H) {
  int64_t o = 0;
  for (int v = L.ny - 1; v >= 0; --v) {
    const int32_t d = decode_y_step(L, v, u);
    o += (int64_t)H.w[v] * (d < 0 ? -(int64_t)d : (int64_t)d);
  }
  return o;
}

// ------------------------------------------------------------ wave helpers
#if defined(__HIPCC__)
__device__ inline uint32_t wave_or(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v |= (uint32_t)__shfl_xor((int)v, off);
  return v;
}
__device__ inline uint32_t wave_and(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v &= (uint32_t)__shfl_xor((int)v, off);
  return v;
}
#endif

// ------------------------------------------------------------ workspace meta
struct Meta {
  uint32_t err;           // latched error bits of this call
  uint32_t narrow;        // bit0: all int64 coefficients fit int32; bit1: fit 24-bit signed
  int64_t ntasks;         // dense: number of windows
  int64_t out_count;      // number of result terms (before the capacity check)
  uint32_t seg_flags[2];  // dense: coefficient-range flags of factor A / B
  uint32_t seg_err[2];    // dense: error bits found while sorting factor A / B
  uint32_t plan_done;     // dense: planning workgroups finished
  uint32_t radix_l2;      // grouped hash: level-2 bits for the products actually made
  int64_t task_rows;      // dense: cost of a task (work items plus window overheads)
  int64_t pad;
  // hash accumulation grouped by code range
  unsigned long long amax, bmax;   // largest |coefficient| of A and of B (int64)
  int64_t nbins;          // bins of all ranges
  int64_t entries;        // products written (grouped entries)
  uint32_t pack;          // entries packed in 8 bytes (value above the hash bits)
  uint32_t reserve;       // each range's terms go to its own entry slots (no shared counter)
};

// Status block owned by a context (device memory, 256 bytes).
struct CtxStatus {
  uint32_t err;
  uint32_t pad0;
  unsigned long long inserts;    // hash insertions counted while statistics are on
  unsigned long long probes;     // slots visited beyond the home slot
  unsigned long long overflows;  // bucketed table: insertions that went to the overflow table
  unsigned long long sink[16];   // discard area of the LDS atomic probe
  uint32_t pad[24];
};
static_assert(sizeof(CtxStatus) == 256, "status block is 256 bytes");

// ------------------------------------------------------------ launchers
// codec
hipError_t launch_minmax(int64_t n, int32_t nv, const int32_t* vals, int32_t* out, hipStream_t s);

// Boxes of up to four exponent arrays in one launch; acc (nseg x 2 x
// KP_MAX_VARS, mins then maxes) and done persist between launches and must
// hold INT_MAX / INT_MIN and 0 before the first one.
// Host-coherent pinned block through which kernels hand small results to a
// host thread that spins on a sequence number (no stream synchronisation).
// Factor boxes come back as partial boxes, one per workgroup of the box
// kernel (at most BOX_PARTS per array); every word carries the low 32 bits
// of the call's sequence number above the value, so the host knows when
// all have arrived without a fence or a cross-workgroup step on the device.
constexpr int BOX_PARTS = 64;
struct Mailbox {
  // per array and box workgroup: KP_MAX_VARS mins, then maxes, tagged
  uint64_t box_part[4][BOX_PARTS][2 * KP_MAX_VARS];
  // a multiply's result count (or -status), low and high halves, and the
  // context's latched status bits, tagged the same way
  uint64_t n_tag[3];
};

#if defined(__HIPCC__)
// Posts a result count and status bits to the mailbox: three tagged words,
// one store each, no fence (the host takes them once all carry the tag).
__device__ __forceinline__ void post_count(Mailbox* mb, uint64_t seq, int64_t n, uint32_t err) {
  const uint64_t tag = (uint64_t)(uint32_t)seq << 32;
  const uint64_t u = (uint64_t)n;
  __hip_atomic_store(&mb->n_tag[0], tag | (u & 0xffffffffu), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&mb->n_tag[1], tag | (u >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&mb->n_tag[2], tag | err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
#endif

struct BoxArgs {
  const int32_t* vals[4];
  int64_t n[4];
  int32_t nv[4];
  int nseg;
  Mailbox* mb;     // device address of the mailbox
  uint64_t seq;
};
// Workgroups (partial boxes) per array of the box kernel for these arrays.
int box_parts(const BoxArgs& A);
hipError_t launch_boxes(const BoxArgs& A, hipStream_t s);
// Posts *out_n and *ctx_err to the mailbox as tagged words (post_count).
hipError_t launch_post_count(const int64_t* out_n, const uint32_t* ctx_err, Mailbox* mb,
                             uint64_t seq, hipStream_t s);
hipError_t launch_encode2(const DevLayout& LA, const DevLayout& LB, int64_t na, int64_t nb,
                          const int32_t* ax, const int32_t* ay, const uint8_t* at, int64_t* akx,
                          int64_t* aky, const int32_t* bx, const int32_t* by, const uint8_t* bt,
                          int64_t* bkx, int64_t* bky, uint32_t* err, hipStream_t s);
hipError_t launch_decode_n(const DevLayout& L, int poisson, const int64_t* n_dev, int64_t cap,
                           const int64_t* codes, int32_t* x, int32_t* y, uint8_t* t, uint32_t* err,
                           hipStream_t s);
hipError_t launch_encode(const DevLayout& L, int64_t n, const int32_t* x, const int32_t* y,
                         const uint8_t* t, int64_t* kx, int64_t* ky, uint32_t* err, hipStream_t s);
hipError_t launch_decode(const DevLayout& L, int poisson, int64_t n, const int64_t* codes,
                         int32_t* x, int32_t* y, uint8_t* t, uint32_t* err, hipStream_t s);

// misc
hipError_t launch_meta_init(Meta* m, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_finalize(const Meta* m, int64_t out_cap, int64_t* out_n, uint32_t* ctx_err,
                           hipStream_t s);
hipError_t launch_coef_range(const int64_t* a, int64_t na, const int64_t* b, int64_t nb, Meta* m,
                             hipStream_t s);

// A 128-bit two's complement coefficient: low word, then high word (the
// output layout of KP_I128).  Sums are formed with a carry out of the low
// word, so that 64-bit atomic adds can accumulate it.
struct I128 {
  uint64_t lo;
  int64_t hi;
  __host__ __device__ constexpr I128() : lo(0), hi(0) {}
  __host__ __device__ constexpr I128(int v) : lo((uint64_t)(int64_t)v), hi(v < 0 ? -1 : 0) {}
  __host__ __device__ constexpr I128(uint64_t l, int64_t h) : lo(l), hi(h) {}
  __host__ __device__ constexpr bool operator==(const I128& o) const {
    return lo == o.lo && hi == o.hi;
  }
  __host__ __device__ constexpr bool operator!=(const I128& o) const { return !(*this == o); }
};
// Words of one coefficient of a dtype (int64 and fp64: 1, int128: 2).
inline constexpr int coef_words(kp_dtype dt) { return dt == KP_I128 ? 2 : 1; }

// dense Laurent
constexpr int64_t DENSE_MAX_BUCKETS = 32768;   // bucket-sort histogram slots (LDS)
constexpr int64_t DENSE_CHUNK = 2048;          // output segment (codes)
constexpr int64_t DENSE_MAX_WINDOW = 18432;    // LDS slots of one window (8 bytes each)
constexpr int64_t DENSE_DUMMY = 64;            // per-lane discard slots after the window
constexpr size_t DENSE_LDS_BYTES = (DENSE_MAX_WINDOW + DENSE_DUMMY) * 8;
constexpr int64_t DENSE_TILE = 16;             // terms of B per tile (one 16-lane row)
constexpr int64_t DENSE_ITEM_ROWS = 64;        // rows of A per work item
constexpr int64_t DENSE_MAX_CODES = (int64_t)1 << 27;   // codes of a dense key space
int dense_bucket_shift(int64_t maxcode, int64_t n);

struct DensePlan {
  int64_t S;             // window (codes), a multiple of DENSE_CHUNK
  int64_t nwin;          // ceil(nkeys / S)
  int64_t ntiles;        // ceil(nb / DENSE_TILE)
  int64_t nkeys;
  int64_t nchunk;        // ceil(nkeys / DENSE_CHUNK)
  int64_t target_tasks;  // tasks wanted (compute units x tasks per unit)
  int64_t max_tasks;     // upper bound on tasks (= target)
  int64_t min_work;      // row visits below which a window is not split
  int64_t items_cap;     // bound on work items (see dense_items_bound)
  int accumulate;        // 1: every window adds into the HBM accumulator, no compaction
  int shiftA, shiftB;    // bucket widths 2^shift of the factor sorts
  int64_t nbkA, nbkB;    // buckets
  int64_t maxcodeA, maxcodeB;   // largest code of each factor's box
  int32_t block;
};
struct DenseBufs {
  Meta* meta;
  const int64_t* a_keys_in; const int64_t* a_coef_in;
  const int64_t* b_keys_in; const int64_t* b_coef_in;
  int64_t na, nb;
  uint64_t* apk; uint64_t* ac;  // A bucket-sorted: {code, low coefficient word}, coefficient
  uint64_t* bpk; uint64_t* bc;  // B bucket-sorted, same layout
  int32_t* rank_a; int32_t* rank_b;
  int32_t* bstart;              // [nbkA + 1] first row of each bucket of A
  int32_t* bstartB;             // [nbkB + 1] first term of each bucket of B
  int64_t* tmin; int64_t* tmax; // [ntiles] code range of each tile of B
  int64_t* win;                 // [5 * (nwin + 1)]: items, rows, split flag, item base, cost base
  int4* recs;                   // [nwin * ntiles] rows of A visited by each (window, tile)
  uint64_t* items;              // [items_cap] work items
  int32_t* task_w;              // [max_tasks] window of each task
  int32_t* task_begin;          // [max_tasks + 1] first item of each task
  int64_t* dense;               // [nwin * S * cw] accumulator of windows split across tasks
  int64_t* stage_k; int64_t* stage_c;   // [nchunk * DENSE_CHUNK (* cw)] compacted chunks
  int64_t* ccount;              // [nchunk] terms per chunk
  int64_t* coff;                // [nchunk] output offset per chunk
  int64_t* out_k; void* out_c; int64_t out_cap; int64_t* out_n;
  uint32_t* ctx_err;
  hipEvent_t ev0, ev1;   // optional: recorded around the window kernel
  // optional: the output scan also posts the count (or -status) and the
  // status bits to this mailbox, tagged with seq (post_count)
  struct Mailbox* mb;
  uint64_t seq;
  // optional: the output copy writes decoded exponents (int32[n][dec.nx])
  // instead of codes
  int32_t* out_exps;
  DevLayout dec;
  // optional truncation tables (input order) and their bucket-sorted copies
  const int32_t* a_sa_in; const int32_t* b_tb_in;
  int32_t* a_sa; int32_t* b_tb;
};
hipError_t dense_setup();
hipError_t launch_dense_laurent(const DensePlan& P, const DenseBufs& B, kp_dtype dt, hipStream_t s);

// hash Laurent / Poisson
struct HashBufs {
  Meta* meta;
  uint64_t* table;       // cap * 2 words: (key + 1, coef bits); int128: cap * 4 words
                         // (key + 1, low word, high word, unused)
  int64_t cap;           // slots (>= 64)
  int64_t max_probe;
  int64_t* out_k; void* out_c; int64_t out_cap;
  hipEvent_t ev0, ev1;   // optional: recorded around the insert kernel
  unsigned long long* stats;   // optional: {insertions, extra probe steps}
  const int32_t* a_sa;   // optional truncation: slack of A's terms, degree of B's
  const int32_t* b_tb;
};
hipError_t launch_hash_laurent(const HashBufs& H, kp_dtype dt, const int64_t* ak, const void* ac,
                               int64_t na, const int64_t* bk, const void* bc, int64_t nb,
                               int rows, hipStream_t s);
struct PoissonPrep {
  int64_t* ap; int64_t* akx; uint8_t* at;     // A: kx + Wx ky, kx, is_sin
  int64_t* bp; int64_t* bm; int64_t* bkx; uint8_t* bt;  // B: kx + Wx ky, kx - Wx ky, kx, is_sin
  int32_t* ao; int32_t* bo;   // harmonic orders of A's and B's terms (truncated products)
  uint4* ad; uint4* bd;       // or their multipliers as 16 signed bytes (all within +-127)
};
// H: optional harmonic truncation (the orders are then written, from L).
hipError_t launch_poisson_prep(int64_t Wx, const int64_t* ax, const int64_t* ay, const uint8_t* as,
                               int64_t na, const int64_t* bx, const int64_t* by,
                               const uint8_t* bs, int64_t nb, const PoissonPrep& P, hipStream_t s,
                               const DevLayout* L = nullptr, const HarmonicSpec* H = nullptr);
hipError_t launch_hash_poisson(const HashBufs& H, int64_t Wx, const PoissonPrep& P,
                               const double* ac, int64_t na, const double* bc, int64_t nb,
                               int rows, hipStream_t s);
hipError_t launch_hash_compact(const HashBufs& H, kp_dtype dt, hipStream_t s);

// Bucketed table (the paper's layout): nbuckets buckets of m slots at the
// start of H.table, hashed by code mod nbuckets, followed by an overflow
// table of ovcap slots (open addressing); H.cap counts both.
struct BucketGeom {
  int m;
  uint64_t nbuckets;
  FastDiv fN;
  int64_t ovcap;
};
hipError_t launch_hash_laurent_bucket(const HashBufs& H, const BucketGeom& G, kp_dtype dt,
                                      const int64_t* ak, const void* ac, int64_t na,
                                      const int64_t* bk, const void* bc, int64_t nb, int rows,
                                      hipStream_t s);
// Orders the terms of both factors by code mod nbuckets (bins of the
// residue, a counting sort per factor): codes, 8-byte coefficients and the
// optional int32 truncation tables, into the out arrays; rank is scratch of
// na + nb int32.
struct ModOrder {
  const int64_t* k_in[2]; const uint64_t* c_in[2]; const int32_t* t_in[2]; int64_t n[2];
  int64_t* k_out[2]; uint64_t* c_out[2]; int32_t* t_out[2]; int32_t* rank[2];
};
hipError_t launch_mod_order(const ModOrder& O, const BucketGeom& G, hipStream_t s);

// Partitioned hash accumulation: products grouped by hash bits in two
// levels through HBM, each final bin accumulated in an LDS table.
struct RadixArgs {
  const int64_t* ak; const void* ac; int64_t na;   // Laurent: codes, coefficients
  const int64_t* bk; const void* bc; int64_t nb;   // (Poisson: coefficients only)
  int64_t Wx; PoissonPrep P;                       // Poisson combined codes
  int rows;              // rows of A per count / scatter workgroup
  int l1, l2;            // log2 of the level-1 partitions and (at most) level-2 bins per
                         // partition; the bits used are chosen on the device (Meta::radix_l2)
  int64_t nblocks;       // count / scatter workgroups (set by the launcher)
  uint32_t* counts;      // [2^l1][nblocks] products per (partition, workgroup), then offsets
  int64_t* pstart;       // [2^l1 + 1] partition totals, then starts
  int64_t* bstart;       // [2^(l1+l2) + 1] bin starts
  uint4* ent1;           // [products] {code, value bits}, grouped by partition
  uint4* ent2;           // [products] the same, grouped by bin
  Meta* meta;
  int64_t* out_k; void* out_c; int64_t out_cap;
  unsigned long long* stats;
  hipEvent_t ev0, ev1;   // optional: recorded around the whole accumulation
  const int32_t* a_sa;   // optional truncation (Laurent): a pair is generated iff
  const int32_t* b_tb;   // b_tb[j] <= a_sa[i]
  int32_t* out_x;        // optional (Laurent): decoded exponents instead of codes
  DevLayout dec;
  int bin_log = 11;      // log2 of the slots of a bin's LDS table (11, 12 or 13)
  uint16_t* bin1 = nullptr;   // [products] level-2 bin of each entry of ent1
  int32_t* out_y = nullptr;   // optional (Poisson, with out_x and out_t): decoded
  uint8_t* out_t = nullptr;   // trigonometric exponents and sin flags instead of keys
  // optional (Poisson): truncation by harmonic order; a pair whose factors'
  // orders (P.ao, P.bo) differ by more than the limit makes no piece, and the
  // bins drop the terms over it (dec decodes the keys)
  int32_t harm_on = 0;
  HarmonicSpec harm{};
  // with P.ad / P.bd: each piece's order is computed from the factors'
  // multipliers and a piece over the limit is never formed
  int32_t harm_exact = 0;
};
// kind: 0 Laurent int64, 1 Laurent fp64, 2 Poisson (fp64), 3 Laurent int64
// factors with exact 128-bit sums (entries carry the pair's indices, the bins
// form the products; the planner caps the tables at 4096 slots).
hipError_t launch_radix(const RadixArgs& R, int kind, hipStream_t s);
// Threads (terms of B) per count / scatter workgroup; the workspace planner
// sizes the per-workgroup histograms with it.
constexpr int RADIX_THREADS = 1024;

// Hash accumulation grouped by output code range (Laurent, int64 or fp64).
// Range r holds the product codes [r << w, (r + 1) << w) of [0, nkeys).  The
// products of a range are found from each row of A and an interval of B
// sorted into buckets of 2^shiftB codes, so nothing is written before they
// are grouped: each product goes once to a bin of its range, chosen by the
// top bits of a w-bit hash of its offset in the range, and each bin is
// accumulated in an LDS table.
struct RangeArgs {
  Meta* meta;
  const int64_t* ak; const void* ac; int64_t na; int64_t maxA;   // A, input order
  const int64_t* bk_in; const void* bc_in; int64_t nb; int64_t maxB;
  const int32_t* a_sa; const int32_t* b_tb_in;   // optional truncation: keep b_tb[j] <= a_sa[i]
  int64_t* bk; uint64_t* bc; int32_t* b_tb;      // B bucket-sorted (b_tb only with truncation)
  int32_t* brank; int32_t* bstart;               // [nb], [nbkB + 1]
  int shiftB; int64_t nbkB;
  int64_t nkeys; int w; int64_t nr;              // ranges of 2^w codes, nr of them
  uint64_t mult, inv;                            // odd multiplier mod 2^w and its inverse
  int64_t nsplit, rows;                          // row splits of A, rows per split (bounds)
  int64_t split_cap;                             // at most this many splits of one range
  int64_t target;                                // products wanted per bin
  int max_l2;                                    // at most 2^max_l2 bins per range
  int64_t nbins_max;
  int64_t* rcount;   // [nr] product bound per range (bucket granularity)
  int32_t* rnb;      // [nr] bins of each range
  int64_t* rbin0;    // [nr + 1] first bin of each range
  int64_t* rtotal;   // [nr] entries of each range
  int64_t* rbase;    // [nr] first entry (and first result slot) of each range
  int64_t* rhole;    // [nr + 1] empty slots below the result count, per range, then prefix
  int64_t* rabove;   // [nr + 1] terms at the result count or beyond, per range, then prefix
  int32_t* rns;      // [nr] row splits of each range (its share of the products)
  int64_t* rupre;    // [nr + 1] first (range, split) unit of each range
  int64_t* rcbase;   // [nr + 1] first count of each range: its bins times its splits
  int32_t* umap;     // [nr * split_cap] range of each (range, split) unit
  int64_t* cnt;      // [nbins_max * split_cap] entries per (bin, split), then offsets in the range
  int32_t* bin_range;  // [nbins_max]
  int64_t* bin_start;  // [nbins_max + 1] first entry of each bin (absolute once scattered)
  int64_t* bin_terms;  // [nbins_max] result terms of each bin
  int64_t* bhole;      // [nbins_max] prefix of the bins' empty slots below the count, in a range
  int64_t* babove;     // [nbins_max] prefix of the bins' terms past the count, in a range
  void* ent;         // entries: 8 bytes (packed) or 16 bytes each
  int64_t* out_k; void* out_c; int64_t out_cap;
  int32_t* out_x; DevLayout dec;   // optional decoded output instead of codes
  hipEvent_t ev0, ev1;
  int bin_log;       // log2 of a bin table's slots (11, 12 or 13)
  unsigned long long* stats;   // optional: {insertions, extra probe steps}
};
hipError_t range_setup();
hipError_t launch_range(const RangeArgs& R, kp_dtype dt, hipStream_t s);

// packed batches (kp_pack.hip): many whole Laurent products in one fixed
// sequence of persistent launches that read a device task table
constexpr int PACK_BLOCK = 256;
struct PackTask {
  DevLayout la, lb;                 // A's and B's code maps; the product's decode
  const int32_t* ax;                // exponents [na][nx], [nb][nx]
  const int32_t* bx;
  const void* ac;                   // coefficients (int64 or double)
  const void* bc;
  int64_t na, nb;
  int64_t* ak;                      // codes (arena)
  int64_t* bk;
  uint64_t* table;                  // direct: one word per code; hash: (code + 1, value) pairs
  int64_t slots;                    // direct: codes; hash: a power of two
  int64_t rows;                     // rows of A per multiply unit
  int64_t bblocks;                  // blocks of PACK_BLOCK terms of B
  int32_t direct, f64;
  int32_t* out_x;                   // [out_cap][nx]
  void* out_c;                      // [out_cap]
  int64_t out_cap;
  unsigned long long* count;        // arena
};
// The table: this header, then three unit prefixes of max_tasks + 1 words
// (prep, multiply, compaction), then max_tasks tasks.
struct PackHeader {
  int32_t ntasks, max_tasks;
  uint32_t err;
  uint32_t pad;
  uint64_t seq;                     // tag of this run's posts
  uint64_t* post;                   // host-mapped: two tagged words per task
};
size_t pack_table_bytes(int max_tasks);
hipError_t launch_pack_boxes(const int32_t* const* vals, const int64_t* n, const int32_t* nv,
                             int nseg, uint64_t* post_dev, uint64_t seq, hipStream_t s);
hipError_t launch_pack_run(void* table_dev, int grid, hipStream_t s);

// diagnostics (kp_diag.hip)
hipError_t probe_lds_atomic(int pattern, int blocks, int iters, unsigned long long* sink,
                            float* ms, hipStream_t s);

// dense Poisson (kp_poisson.hip)
hipError_t launch_poisson_dense_prep(int64_t Wx, int64_t N, int64_t Hya, int64_t Hyb,
                                     const int64_t* ax, const int64_t* ay, const uint8_t* as,
                                     const double* ac, int64_t na, const int64_t* bx,
                                     const int64_t* by, const uint8_t* bs, const double* bc,
                                     int64_t nb, int64_t* a_codes, double* a_coef,
                                     int64_t* b_codes, double* b_coef, hipStream_t s);
hipError_t launch_poisson_fold(int64_t Wx, int64_t Hy, int64_t N, const double* acc, Meta* meta,
                               int64_t* out_k, double* out_c, int64_t out_cap, hipStream_t s);

}  // namespace kp
