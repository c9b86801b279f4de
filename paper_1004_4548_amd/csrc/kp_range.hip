// kp_range.hip -- hash accumulation of highly sparse Laurent products,
// grouped by output code range.
//
// Section 3.2 accumulates the products of a highly sparse multiplication in a
// hash table keyed by the product's code.  Here the table is split twice so
// that every part of it lives in LDS.  The code space [0, nkeys) is cut into
// ranges of 2^w consecutive codes; since B is sorted by code (into buckets of
// 2^shiftB codes), the products of row i of A that fall in range r are the
// terms of one interval of B (Section 3: the schoolbook product of the coded
// factors, restricted to an output interval, as Section 4 restricts threads
// to disjoint output intervals).  Nothing is written before grouping: each
// product is formed from the factors, hashed within its range (an odd
// multiplier modulo 2^w, a bijection, so the hash identifies the code), and
// written once to a bin of its range, the bin being the top bits of the
// hash.  One workgroup then accumulates each bin in an LDS open-addressing
// table and writes its nonzero terms.
//
// HBM traffic per product is one entry written and read (8 bytes when the
// value fits above the w hash bits, else 16), instead of a 16-byte table slot
// read and written back per product in a global table.
//
// Result slots: the entries of each bin occupy a run of entry positions, and
// the bin's terms (at most its entries) are written to the first slots of
// that run.  The count N of all terms is then known, and the few terms that
// lie at N or beyond are moved into the empty slots below N, so the result
// is contiguous without a counter shared by all bins.  When the entries
// would not fit the caller's capacity, one shared counter places the terms
// instead.
//
// A bin with more distinct codes than its table holds (possible only for
// adversarial codes, since bins are sized from the product counts) is redone
// on halves of its hash interval until each part fits: an interval of at most
// as many hash values as slots always fits, the hash being a bijection.
#include <climits>
#include <type_traits>

#include "kp_internal.h"

namespace kp {

namespace {

constexpr uint64_t GOLD = 0x9E3779B97F4A7C15ull;   // 2^64 / golden ratio (Fibonacci hashing)
constexpr int RG_BLOCK = 1024;    // threads of the counting and scatter workgroups
constexpr int RG_MAX_L2 = 10;     // at most 1024 bins per range
constexpr int SORT_BLOCK = 1024;
constexpr int SMALL_BLOCK = 256;
constexpr int BIN_PER = 8;        // entries per thread loaded at once in a bin (slots / threads)
constexpr int STACK = 72;         // hash intervals of a bin's overflow passes (depth <= 62)

__device__ __forceinline__ uint64_t uabs(int64_t c) {
  return c < 0 ? 0ull - (uint64_t)c : (uint64_t)c;
}

__device__ __forceinline__ int64_t mul_value(int64_t a, int64_t b) {
  return (int64_t)((uint64_t)a * (uint64_t)b);   // wraps modulo 2^64
}
__device__ __forceinline__ double mul_value(double a, double b) { return a * b; }

template <typename T>
__device__ __forceinline__ T from_bits(uint64_t u) {
  T v;
  __builtin_memcpy(&v, &u, 8);
  return v;
}
template <typename T>
__device__ __forceinline__ uint64_t to_bits(T v) {
  uint64_t u;
  __builtin_memcpy(&u, &v, 8);
  return u;
}

__device__ __forceinline__ uint64_t wmask(int w) {
  return w >= 64 ? ~0ull : ((1ull << w) - 1);
}

// Interval [j0, j1) of bucket-sorted B holding every term b with a + b in
// [lo, hi) (and a few neighbours of the edge buckets); false when empty.
__device__ __forceinline__ bool row_interval(const RangeArgs& R, int64_t a, int64_t lo,
                                             int64_t hi, int64_t* j0, int64_t* j1) {
  int64_t xlo = lo - a, xhi = hi - 1 - a;
  if (xhi < 0 || xlo > R.maxB) return false;
  xlo = xlo < 0 ? 0 : xlo;
  xhi = xhi > R.maxB ? R.maxB : xhi;
  *j0 = R.bstart[xlo >> R.shiftB];
  *j1 = R.bstart[(xhi >> R.shiftB) + 1];
  return *j0 < *j1;
}

// Bin of hash h among nb bins of its range: floor(h nb / 2^w), so that every
// bin of a range covers an equal share of the hash values.
__device__ __forceinline__ uint32_t bin_of(uint64_t h, int w, uint32_t nb) {
  return w ? (uint32_t)__umul64hi(h << (64 - w), (uint64_t)nb) : 0u;
}

// Exclusive scan of one value per thread over a workgroup of NT threads.
template <int NT, typename V>
__device__ __forceinline__ V block_scan(V v, V* s_ws, V* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  V incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const V y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) s_ws[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    V run = 0;
    for (int k = 0; k < NT / 64; ++k) {
      const V x = s_ws[k];
      s_ws[k] = run;
      run += x;
    }
    s_ws[NT / 64] = run;
  }
  __syncthreads();
  const V r = s_ws[wave] + incl - v;
  *total = s_ws[NT / 64];
  __syncthreads();
  return r;
}

// Exclusive scan, in place, of a[0..n) by one workgroup of NT threads, each
// taking a contiguous run; returns the total.
template <int NT, typename V>
__device__ V block_scan_runs(V* a, int64_t n) {
  __shared__ V s_ws[NT / 64 + 1];
  const int64_t per = (n + NT - 1) / NT;
  const int64_t r0 = min(n, (int64_t)threadIdx.x * per), r1 = min(n, r0 + per);
  V local = 0;
  for (int64_t k = r0; k < r1; ++k) local += a[k];
  V total;
  V run = block_scan<NT, V>(local, s_ws, &total);
  for (int64_t k = r0; k < r1; ++k) {
    const V x = a[k];
    a[k] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

template <int NT, typename V, typename Op>
__device__ V block_reduce(V v, Op op) {
  __shared__ V s_red[NT / 64];
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  V r = s_red[0];
  for (int k = 1; k < NT / 64; ++k) r = op(r, s_red[k]);
  __syncthreads();
  return r;
}

// ------------------------------------------------------------ B by buckets
// One workgroup: bucket histogram of B's codes, each term's rank in its
// bucket, bucket starts; also clears the per-range counters of this call and
// finds B's largest |coefficient|.
template <typename T>
__global__ void __launch_bounds__(SORT_BLOCK) k_rg_bsort(RangeArgs R) {
  extern __shared__ int32_t hist[];
  const int tid = threadIdx.x;
  for (int64_t k = tid; k < R.nbkB; k += SORT_BLOCK) hist[k] = 0;
  for (int64_t r = tid; r < R.nr; r += SORT_BLOCK) R.rcount[r] = 0;
  __syncthreads();
  uint64_t mx = 0;
  uint32_t err = 0;
  for (int64_t j = tid; j < R.nb; j += SORT_BLOCK) {
    int64_t c = R.bk_in[j];
    if (c < 0 || c > R.maxB) {
      err |= ERR_RANGE;
      c = c < 0 ? 0 : R.maxB;
    }
    R.brank[j] = atomicAdd(&hist[c >> R.shiftB], 1);
    if constexpr (std::is_same<T, int64_t>::value)
      mx = max(mx, uabs(static_cast<const int64_t*>(R.bc_in)[j]));
  }
  __syncthreads();
  const int64_t per = (R.nbkB + SORT_BLOCK - 1) / SORT_BLOCK;
  const int64_t k0 = min(R.nbkB, (int64_t)tid * per), k1 = min(R.nbkB, k0 + per);
  int64_t local = 0;
  for (int64_t k = k0; k < k1; ++k) local += hist[k];
  __shared__ int64_t s_ws[SORT_BLOCK / 64 + 1];
  int64_t total;
  int64_t run = block_scan<SORT_BLOCK, int64_t>(local, s_ws, &total);
  for (int64_t k = k0; k < k1; ++k) {
    R.bstart[k] = (int32_t)run;
    run += hist[k];
  }
  if (tid == 0) R.bstart[R.nbkB] = (int32_t)total;
  mx = block_reduce<SORT_BLOCK>(mx, [](uint64_t x, uint64_t y) { return x > y ? x : y; });
  err = block_reduce<SORT_BLOCK>(err, [](uint32_t x, uint32_t y) { return x | y; });
  if (tid == 0) {
    R.meta->bmax = mx;
    if (err) atomicOr(&R.meta->err, err);
  }
}

__global__ void __launch_bounds__(SMALL_BLOCK) k_rg_bplace(RangeArgs R) {
  const int64_t j = (int64_t)blockIdx.x * SMALL_BLOCK + threadIdx.x;
  if (j >= R.nb) return;
  const int64_t c = R.bk_in[j];
  const int64_t cc = c < 0 ? 0 : c > R.maxB ? R.maxB : c;
  const int64_t at = R.bstart[cc >> R.shiftB] + R.brank[j];
  R.bk[at] = c;
  R.bc[at] = static_cast<const uint64_t*>(R.bc_in)[j];
  if (R.b_tb) R.b_tb[at] = R.b_tb_in[j];
}

// ------------------------------------------------------------ counting
// Products per range, as an upper bound (whole buckets): one workgroup per
// (range, row split).  The first range also checks A's codes and finds A's
// largest |coefficient|.
template <typename T>
__global__ void __launch_bounds__(SMALL_BLOCK) k_rg_count0(RangeArgs R) {
  const int64_t r = blockIdx.x, s = blockIdx.y;
  const int64_t lo = r << R.w, hi = min(R.nkeys, (r + 1) << R.w);
  const int64_t i0 = s * R.rows, i1 = min(R.na, i0 + R.rows);
  int64_t sum = 0;
  uint64_t mx = 0;
  uint32_t err = 0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += SMALL_BLOCK) {
    const int64_t a = R.ak[i];
    if (r == 0) {
      if (a < 0 || a > R.maxA) err |= ERR_RANGE;
      if constexpr (std::is_same<T, int64_t>::value)
        mx = max(mx, uabs(static_cast<const int64_t*>(R.ac)[i]));
    }
    int64_t j0, j1;
    if (row_interval(R, a, lo, hi, &j0, &j1)) sum += j1 - j0;
  }
  sum = block_reduce<SMALL_BLOCK>(sum, [](int64_t x, int64_t y) { return x + y; });
  if (threadIdx.x == 0 && sum)
    atomicAdd(reinterpret_cast<unsigned long long*>(&R.rcount[r]), (unsigned long long)sum);
  if (r == 0) {
    mx = block_reduce<SMALL_BLOCK>(mx, [](uint64_t x, uint64_t y) { return x > y ? x : y; });
    err = block_reduce<SMALL_BLOCK>(err, [](uint32_t x, uint32_t y) { return x | y; });
    if (threadIdx.x == 0) {
      atomicMax(&R.meta->amax, mx);
      if (err) atomicOr(&R.meta->err, err);
    }
  }
}

// One workgroup: the bins of each range (about `target` products each, from
// the range's bound on products), first bin of each range, and whether int64
// entries fit in 8 bytes (every product below 2^(63 - w) in size).
template <typename T>
__global__ void __launch_bounds__(1024) k_rg_plan(RangeArgs R) {
  __shared__ int s_cut;
  const int tid = threadIdx.x;
  if (tid == 0) s_cut = 0;
  __syncthreads();
  const int64_t per = (R.nr + 1023) / 1024;
  const int64_t r0 = min(R.nr, (int64_t)tid * per), r1 = min(R.nr, r0 + per);
  // at most 2^max_l2 bins, and no more bins than hash values
  const int64_t most = min((int64_t)1 << R.max_l2, (int64_t)1 << min(R.w, 30));
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t c = R.rcount[r];
    R.rnb[r] = (int32_t)max((int64_t)1, min(most, (c + R.target - 1) / R.target));
  }
  // half as many bins everywhere while the bins would outgrow their arrays
  int64_t total = 0;
  __shared__ int64_t s_ws[1024 / 64 + 1];
  for (int pass = 0; pass <= RG_MAX_L2; ++pass) {
    int64_t local = 0;
    for (int64_t r = r0; r < r1; ++r) local += max(1, R.rnb[r] >> s_cut);
    int64_t run = block_scan<1024, int64_t>(local, s_ws, &total);
    if (total <= R.nbins_max) {
      for (int64_t r = r0; r < r1; ++r) {
        const int nb = max(1, R.rnb[r] >> s_cut);
        R.rnb[r] = nb;
        R.rbin0[r] = run;
        run += nb;
      }
      break;
    }
    __syncthreads();
    if (tid == 0) ++s_cut;
    __syncthreads();
  }
  // row splits per range in proportion to its products, so that the
  // counting and grouping workgroups get about equal shares (products
  // concentrate in part of the code space for dense-like factors)
  __syncthreads();
  int64_t local = 0;
  for (int64_t r = r0; r < r1; ++r) local += R.rcount[r];
  int64_t all = 0;
  (void)block_scan<1024, int64_t>(local, s_ws, &all);
  const int64_t units = R.nr * R.nsplit;
  const int64_t share = max((int64_t)1, (all + units - 1) / units);
  const int64_t cap = min(R.split_cap, max((int64_t)1, R.na));
  int64_t lu = 0, lc = 0;
  for (int64_t r = r0; r < r1; ++r) {
    // (a range is split once it holds eight times its even share: mild
    // unevenness costs less than the extra walks over the rows)
    const int64_t ns = max((int64_t)1, min(cap, R.rcount[r] / (4 * share)));
    R.rns[r] = (int32_t)ns;
    lu += ns;
    lc += ns * R.rnb[r];
  }
  int64_t tu = 0, tc = 0;
  int64_t ru = block_scan<1024, int64_t>(lu, s_ws, &tu);
  int64_t rc = block_scan<1024, int64_t>(lc, s_ws, &tc);
  for (int64_t r = r0; r < r1; ++r) {
    R.rupre[r] = ru;
    R.rcbase[r] = rc;
    for (int32_t k = 0; k < R.rns[r]; ++k) R.umap[ru + k] = (int32_t)r;
    ru += R.rns[r];
    rc += (int64_t)R.rns[r] * R.rnb[r];
  }
  if (tid == 0) {
    R.rupre[R.nr] = tu;
    R.rcbase[R.nr] = tc;
    R.rbin0[R.nr] = total;
    R.meta->nbins = total;
    uint32_t pack = 0;
    if constexpr (std::is_same<T, int64_t>::value) {
      const uint64_t am = R.meta->amax, bm = R.meta->bmax;
      const uint64_t lim = 1ull << (63 - R.w);
      pack = (__umul64hi(am, bm) == 0 && am * bm < lim) ? 1u : 0u;
    }
    R.meta->pack = pack;
  }
}

// ------------------------------------------------------------ expansion
// A wavefront takes rows of A 64 at a time (lane l holds one row): the rows'
// intervals of B are found together, their lengths scanned, and the row data
// staged in LDS.  The candidates of the 64 rows are then taken 64 at a time,
// lane l holding candidate k = base + l: its row m is the last with
// pre[m] <= k (a binary search over the staged prefix), its term of B is
// jb[m] + k.  Every lane has work and the loads of B are coalesced, whatever
// the rows' interval lengths.
constexpr int WAVES = RG_BLOCK / 64;

struct WaveRows {
  int32_t pre[65];    // exclusive prefix of the rows' interval lengths; pre[64] = total
  int32_t sa[64];     // truncation slack of each row
  int64_t jb[64];     // first term of B of row m, minus pre[m]
  int64_t a[64];      // code of row m
  uint64_t ca[64];    // coefficient bits of row m
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront's walk over its batches of rows in (range, split).
template <typename T>
struct WaveWalk {
  int64_t row0, row1;   // rows of the split
  int64_t lo, hi;       // the range's codes
  int64_t bt;           // current batch (rows row0 + 64 bt ..)
  int32_t kb, total;    // next candidate and candidates of the batch
  bool done;

  __device__ __forceinline__ void start(int64_t r0, int64_t r1, int64_t l, int64_t h, int wave) {
    row0 = r0;
    row1 = r1;
    lo = l;
    hi = h;
    bt = wave - WAVES;
    kb = total = 0;
    done = false;
  }
  // Stages the next batch with at least one candidate (or sets done).
  __device__ __forceinline__ void next_batch(const RangeArgs& R, WaveRows& W) {
    const int lane = threadIdx.x & 63;
    for (;;) {
      bt += WAVES;
      const int64_t first = row0 + 64 * bt;
      if (first >= row1) {
        done = true;
        return;
      }
      const int64_t i = first + lane;
      int64_t j0 = 0, j1 = 0, a = 0;
      uint64_t ca = 0;
      int32_t sa = INT_MAX;
      if (i < row1) {
        a = R.ak[i];
        if (row_interval(R, a, lo, hi, &j0, &j1)) {
          ca = static_cast<const uint64_t*>(R.ac)[i];
          if (R.a_sa) sa = R.a_sa[i];
        } else {
          j0 = j1 = 0;
        }
      }
      const int32_t cnt = (int32_t)(j1 - j0);
      int32_t incl = cnt;
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
      }
      const int32_t excl = incl - cnt;
      const int32_t tot = __shfl(incl, 63);
      wave_sync();
      W.pre[lane] = excl;
      if (lane == 63) W.pre[64] = tot;
      W.jb[lane] = j0 - excl;
      W.a[lane] = a;
      W.ca[lane] = ca;
      W.sa[lane] = sa;
      wave_sync();
      if (tot > 0) {
        kb = 0;
        total = tot;
        return;
      }
    }
  }
  // The lane's candidate of the next 64: false once the walk is over (for
  // the whole wavefront); *ok tells whether the lane holds a product of the
  // range (code in range, kept by the truncation).  A product whose value is
  // zero is kept too, so that counting needs no coefficients (its sum is
  // dropped with the other zero sums); VAL: form the value.
  template <bool VAL>
  __device__ __forceinline__ bool step(const RangeArgs& R, WaveRows& W, int w, uint64_t mult,
                                       bool* ok, uint64_t* h, T* v) {
    if (!done && kb >= total) next_batch(R, W);
    if (done) return false;
    const int32_t k = kb + (threadIdx.x & 63);
    kb += 64;
    *ok = false;
    if (k >= total) return true;
    int m = 0, z = 64;   // pre[m] <= k < pre[z]
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int mid = (m + z) >> 1;
      if (W.pre[mid] <= k) m = mid;
      else z = mid;
    }
    const int64_t j = W.jb[m] + k;
    const int64_t c = W.a[m] + R.bk[j];
    if (c < lo || c >= hi) return true;
    if (R.b_tb && R.b_tb[j] > W.sa[m]) return true;
    if (VAL) *v = mul_value(from_bits<T>(W.ca[m]), from_bits<T>(R.bc[j]));
    *h = ((uint64_t)(c - lo) * mult) & wmask(w);
    *ok = true;
    return true;
  }
};

// The (range, split) unit of workgroup g: false past the last unit.  Split s
// of range r takes rows [s ceil(na / ns), ...) of A, ns its range's splits.
struct Unit {
  int64_t r, s, ns, i0, i1;
};
__device__ __forceinline__ bool unit_of(const RangeArgs& R, int64_t g, Unit* u) {
  if (g >= R.rupre[R.nr]) return false;
  const int64_t a = R.umap[g];
  u->r = a;
  u->s = g - R.rupre[a];
  u->ns = R.rns[a];
  const int64_t rows = (R.na + u->ns - 1) / u->ns;
  u->i0 = u->s * rows;
  u->i1 = min(R.na, u->i0 + rows);
  return true;
}

// Entries per (bin, split) of each range.
template <typename T>
__global__ void __launch_bounds__(RG_BLOCK, 8) k_rg_count1(RangeArgs R) {   // two per CU
  __shared__ uint32_t hist[1 << RG_MAX_L2];
  __shared__ WaveRows rows[WAVES];
  // the grid walks the (range, split) units
  for (int64_t gu = blockIdx.x;; gu += gridDim.x) {
    Unit U;
    if (!unit_of(R, gu, &U)) return;
    const int64_t r = U.r, s = U.s;
    const uint32_t nbin = (uint32_t)R.rnb[r];
    for (int k = threadIdx.x; k < (int)nbin; k += RG_BLOCK) hist[k] = 0;
    __syncthreads();
    const int64_t lo = r << R.w, hi = min(R.nkeys, (r + 1) << R.w);
    const int wave = threadIdx.x >> 6;
    WaveWalk<T> g;
    g.start(U.i0, U.i1, lo, hi, wave);
    bool ok;
    uint64_t h = 0;
    T v{};
    while (g.template step<false>(R, rows[wave], R.w, R.mult, &ok, &h, &v))
      if (ok) atomicAdd(&hist[bin_of(h, R.w, nbin)], 1u);
    __syncthreads();
    int64_t* c = R.cnt + R.rcbase[r];
    for (int k = threadIdx.x; k < (int)nbin; k += RG_BLOCK) c[k * U.ns + s] = hist[k];
    __syncthreads();   // the next unit clears hist
  }
}

// One workgroup per range: offsets of every (bin, split) within the range,
// each bin's first entry (within the range) and range, and the range's
// entries.
__global__ void __launch_bounds__(1024) k_rg_scan1(RangeArgs R) {
  const int64_t r = blockIdx.x;
  const int64_t b0 = R.rbin0[r], nbin = R.rbin0[r + 1] - b0;
  const int64_t ns = R.rns[r];
  int64_t* c = R.cnt + R.rcbase[r];
  const int64_t total = block_scan_runs<1024, int64_t>(c, nbin * ns);
  for (int64_t k = threadIdx.x; k < nbin; k += 1024) {
    R.bin_start[b0 + k] = c[k * ns];   // within the range; made absolute by the scatter
    R.bin_range[b0 + k] = (int32_t)r;
  }
  if (threadIdx.x == 0) R.rtotal[r] = total;
}

// One workgroup: first entry of each range, the number of entries, and
// whether the result terms can take the entry slots of their bins.
__global__ void __launch_bounds__(1024) k_rg_scan2(RangeArgs R) {
  const int64_t per = (R.nr + 1023) / 1024;
  const int64_t r0 = min(R.nr, (int64_t)threadIdx.x * per), r1 = min(R.nr, r0 + per);
  int64_t local = 0;
  for (int64_t r = r0; r < r1; ++r) local += R.rtotal[r];
  __shared__ int64_t s_ws[1024 / 64 + 1];
  int64_t total;
  int64_t run = block_scan<1024, int64_t>(local, s_ws, &total);
  for (int64_t r = r0; r < r1; ++r) {
    R.rbase[r] = run;
    run += R.rtotal[r];
  }
  if (threadIdx.x == 0) {
    R.meta->entries = total;
    R.meta->reserve = total <= R.out_cap ? 1u : 0u;
    R.bin_start[R.meta->nbins] = total;
  }
}

// ------------------------------------------------------------ grouping
// The products of (range r, rows of split s), STEPS candidates per lane per
// chunk: each chunk is counting-sorted by bin through LDS and written as
// contiguous runs after this workgroup's earlier runs in each bin.  The
// 8-byte entry form is staged as it is written, twelve candidates per lane
// per chunk; the 16-byte form six, in the same 96 KiB of LDS.
constexpr int RG_STAGE_BYTES = RG_BLOCK * 96;

struct ScatterLds {
  uint4 stage[RG_STAGE_BYTES / 16];
  WaveRows rows[WAVES];
  int64_t base[1 << RG_MAX_L2];
  uint32_t coff[1 << RG_MAX_L2];
  uint32_t s_ws[RG_BLOCK / 64 + 1];
};

template <typename T, bool PACK>
__device__ __forceinline__ void scatter_unit(const RangeArgs& R, const Unit& U, ScatterLds& L) {
  constexpr int STEPS = PACK ? 12 : 6;
  static_assert(RG_BLOCK * STEPS * (PACK ? 8 : 16) == RG_STAGE_BYTES, "stage size");
  uint64_t* stage8 = reinterpret_cast<uint64_t*>(L.stage);
  const int tid = threadIdx.x, wave = tid >> 6;
  const int64_t r = U.r, s = U.s;
  const int nbin = R.rnb[r];
  const int w = R.w;
  const uint64_t mult = R.mult, mw = wmask(w);
  const int64_t b0 = R.rbin0[r], rb = R.rbase[r];
  for (int k = tid; k < nbin; k += RG_BLOCK) {
    L.base[k] = rb + R.cnt[R.rcbase[r] + k * U.ns + s];
    L.coff[k] = 0;
    if (s == 0) R.bin_start[b0 + k] += rb;   // the bins' first entries, absolute
  }
  __syncthreads();
  const int64_t lo = r << w, hi = min(R.nkeys, (r + 1) << w);
  WaveWalk<T> g;
  g.start(U.i0, U.i1, lo, hi, wave);
  uint64_t* ent8 = static_cast<uint64_t*>(R.ent);
  uint4* ent16 = static_cast<uint4*>(R.ent);
  for (;;) {
    uint64_t hh[STEPS], vb[STEPS];   // PACK: hh holds the packed entry
    uint32_t bn[STEPS], rank[STEPS];
    uint32_t mask = 0;
#pragma unroll
    for (int u = 0; u < STEPS; ++u) {
      bool ok = false;
      uint64_t h = 0;
      T v{};
      if (!g.template step<true>(R, L.rows[wave], w, mult, &ok, &h, &v)) break;
      if (!ok) continue;
      if (PACK) {
        hh[u] = (to_bits(v) << w) | h;
      } else {
        hh[u] = h;
        vb[u] = to_bits(v);
      }
      bn[u] = bin_of(h, w, (uint32_t)nbin);
      rank[u] = atomicAdd(&L.coff[bn[u]], 1u);
      mask |= 1u << u;
    }
    __syncthreads();
    const uint32_t mine = tid < nbin ? L.coff[tid] : 0u;
    uint32_t total;
    const uint32_t off = block_scan<RG_BLOCK, uint32_t>(mine, L.s_ws, &total);
    if (tid < nbin) L.coff[tid] = off;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < STEPS; ++u)
      if ((mask >> u) & 1u) {
        const uint32_t at = L.coff[bn[u]] + rank[u];
        if (PACK)
          stage8[at] = hh[u];
        else
          L.stage[at] = make_uint4((uint32_t)hh[u], (uint32_t)(hh[u] >> 32), (uint32_t)vb[u],
                                   (uint32_t)(vb[u] >> 32));
      }
    __syncthreads();
    for (uint32_t t = tid; t < total; t += RG_BLOCK) {
      if (PACK) {
        const uint64_t e = stage8[t];
        const uint32_t k = bin_of(e & mw, w, (uint32_t)nbin);
        ent8[L.base[k] + (t - L.coff[k])] = e;
      } else {
        const uint4 e = L.stage[t];
        const uint32_t k = bin_of(((uint64_t)e.y << 32) | e.x, w, (uint32_t)nbin);
        ent16[L.base[k] + (t - L.coff[k])] = e;
      }
    }
    __syncthreads();
    if (tid < nbin) {
      L.base[tid] += mine;
      L.coff[tid] = 0;
    }
    if (!__syncthreads_or(!g.done)) break;
  }
  __syncthreads();   // the next unit resets base and coff
}

template <typename T>
__global__ void __launch_bounds__(RG_BLOCK) k_rg_scatter(RangeArgs R) {
  __shared__ ScatterLds L;
  const bool pack = R.meta->pack != 0;
  // the grid walks the (range, split) units
  for (int64_t gu = blockIdx.x;; gu += gridDim.x) {
    Unit U;
    if (!unit_of(R, gu, &U)) return;
    if constexpr (std::is_same<T, int64_t>::value) {   // only int64 entries are packed
      if (pack)
        scatter_unit<T, true>(R, U, L);
      else
        scatter_unit<T, false>(R, U, L);
    } else {
      scatter_unit<T, false>(R, U, L);
    }
  }
}

// ------------------------------------------------------------ bins
__device__ __forceinline__ void lds_add(int64_t* p, int64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}
__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }

// Entry k: its hash and value, from the 8-byte packed form (value above the
// w hash bits) or the 16-byte one.
// The load takes 16 bytes at a stride of 8 or 16 whatever the form (no branch
// around it, so that a thread's loads are all in flight together; the 8
// bytes past a packed entry lie inside the entry array, which is sized for
// 16-byte entries).
template <typename T>
__device__ __forceinline__ void entry_at(const RangeArgs& R, bool pack, int w, int64_t k,
                                         uint64_t* h, T* v) {
  const uint4 e = *reinterpret_cast<const uint4*>(static_cast<const char*>(R.ent) +
                                                  k * (pack ? 8 : 16));
  const uint64_t lo64 = ((uint64_t)e.y << 32) | e.x;
  if (pack) {
    *h = lo64 & wmask(w);
    *v = from_bits<T>((uint64_t)((int64_t)lo64 >> w));
  } else {
    *h = lo64;
    *v = from_bits<T>(((uint64_t)e.w << 32) | e.z);
  }
}

// One workgroup per bin: the bin's entries go into an LDS table (key = hash
// + 1, linear probing from a second hash of the key); the table is compacted
// in LDS and the nonzero terms are written one per thread with every lane
// busy, from the bin's first entry slot on (the slots of its entries) or,
// when the entries outnumber the result slots, at an offset taken from the
// call's counter.
template <typename T, int LOG>
__global__ void __launch_bounds__((1 << LOG) / BIN_PER) k_rg_bins(RangeArgs R) {
  using K = unsigned long long;
  constexpr int SLOTS = 1 << LOG, NT = SLOTS / BIN_PER;
  __shared__ K keys[SLOTS];
  __shared__ uint64_t vwords[SLOTS];
  T* vals = reinterpret_cast<T*>(vwords);
  __shared__ int64_t s_wave[NT / 64];
  __shared__ int64_t s_base;
  __shared__ int s_over, s_sp;
  __shared__ unsigned long long s_lo[STACK], s_hi[STACK];
  const int64_t b = blockIdx.x;
  if (b >= R.meta->nbins) return;
  const int64_t s = R.bin_start[b], e = R.bin_start[b + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (s == e) {
    if (tid == 0) R.bin_terms[b] = 0;
    return;
  }
  const int w = R.w;
  const bool pack = R.meta->pack != 0;
  const bool reserve = R.meta->reserve != 0;
  const int64_t lo = (int64_t)R.bin_range[b] << w;
  // the bin's first BIN_PER entries per thread, loaded at once: the rounds
  // that reach into the bin (a branch on the bin's size, the same for every
  // thread), indices past the bin repeating its last entry, unused; packed
  // entries are read as their 8 bytes
  uint64_t h0[BIN_PER];
  T v0[BIN_PER];
  bool packed_load = false;
  if constexpr (std::is_same<T, int64_t>::value) {
    if (pack) {
      packed_load = true;
      const uint64_t* ent8 = static_cast<const uint64_t*>(R.ent);
      const uint64_t mw0 = wmask(w);
#pragma unroll
      for (int u = 0; u < BIN_PER; ++u)
        if (s + (int64_t)u * NT < e) {
          const uint64_t x = ent8[min(s + tid + (int64_t)u * NT, e - 1)];
          h0[u] = x & mw0;
          v0[u] = (int64_t)x >> w;
        }
    }
  }
  if (!packed_load) {
#pragma unroll
    for (int u = 0; u < BIN_PER; ++u)
      if (s + (int64_t)u * NT < e)
        entry_at(R, pack, w, min(s + tid + (int64_t)u * NT, e - 1), &h0[u], &v0[u]);
  }
  for (int i = tid; i < SLOTS; i += NT) {
    keys[i] = 0;
    vals[i] = T(0);
  }
  if (tid == 0) s_over = 0;
  __syncthreads();
  int64_t ins = 0, extra = 0;
  const bool stats = R.stats != nullptr;
  // inserts (h, v) when h lies in [ilo, ihi]; a full table sets s_over.  The
  // probe loop has one exit test, and the value is added once the slot is
  // found, so a wavefront's lanes leave the loop with little mask handling.
  const auto insert = [&](uint64_t h, T v, uint64_t ilo, uint64_t ihi) {
    if (h < ilo || h > ihi) return;
    const K key = (K)(h + 1);
    uint32_t slot = (uint32_t)((h * GOLD) >> (64 - LOG));
    // one compare-and-swap claims an empty slot or returns its key
    K c = atomicCAS(&keys[slot], (K)0, key);
    int q = 0;
#pragma nounroll
    while (c != 0 && c != key && q < SLOTS - 1) {
      ++q;
      slot = (slot + 1) & (SLOTS - 1);
      c = atomicCAS(&keys[slot], (K)0, key);
    }
    if (c != 0 && c != key) {   // every slot holds another code
      s_over = 1;
      return;
    }
    lds_add(&vals[slot], v);
    if (stats) {
      ++ins;
      extra += q;
    }
  };
  T* out_c = static_cast<T*>(R.out_c);
  const int nx = R.dec.nx;
  const bool pairs = (nx & 1) == 0 && ((uintptr_t)R.out_x & 7) == 0;
  const uint64_t inv = R.inv, mw = wmask(w);
  // compacts the table, writes its nonzero terms after the `done` already
  // written for this bin, leaves the table cleared when asked (another hash
  // interval of the bin follows); returns the count
  const auto emit = [&](int64_t done, bool clear) -> int64_t {
    K kk[BIN_PER];
    T vv[BIN_PER];
    uint64_t ball[BIN_PER];
    int64_t cnt = 0;
#pragma unroll
    for (int u = 0; u < BIN_PER; ++u) {
      const int i = u * NT + tid;
      kk[u] = keys[i];
      vv[u] = vals[i];
      ball[u] = __ballot(kk[u] != 0 && vv[u] != T(0));
      cnt += __popcll(ball[u]);
    }
    if (lane == 0) s_wave[wave] = cnt;
    __syncthreads();
    int64_t tot = 0, pos = 0;
    for (int k = 0; k < NT / 64; ++k) {
      if (k == wave) pos = tot;
      tot += s_wave[k];
    }
    if (!reserve && tid == 0)
      s_base = tot ? (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(&R.meta->out_count),
                                        (unsigned long long)tot)
                   : 0;
    const uint64_t lt = (1ull << lane) - 1;
#pragma unroll
    for (int u = 0; u < BIN_PER; ++u) {
      if (ball[u] & (1ull << lane)) {
        const int64_t q = pos + __popcll(ball[u] & lt);
        keys[q] = kk[u];
        vals[q] = vv[u];
      }
      pos += __popcll(ball[u]);
    }
    __syncthreads();
    const int64_t base = reserve ? s + done : s_base;
    const int64_t m = min(tot, R.out_cap - base);
    for (int64_t t = tid; t < m; t += NT) {
      const int64_t q = base + t;
      const uint64_t code = (uint64_t)lo + ((((uint64_t)keys[t] - 1) * inv) & mw);
      if (R.out_x) {
        uint64_t c = code;
        if (pairs) {
          int2* o = reinterpret_cast<int2*>(R.out_x + q * nx);
          for (int v = 0; v < nx; v += 2) {
            const int32_t x0 = decode_step_fast(R.dec, v, c);
            o[v >> 1] = make_int2(x0, decode_step_fast(R.dec, v + 1, c));
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
      for (int i = tid; i < SLOTS; i += NT) {
        keys[i] = 0;
        vals[i] = T(0);
      }
      __syncthreads();
    }
    return tot;
  };
#pragma unroll
  for (int u = 0; u < BIN_PER; ++u)
    if (s + tid + (int64_t)u * NT < e) insert(h0[u], v0[u], 0, ~0ull);
  // bins of many products per code can hold more entries than slots
  for (int64_t k = s + tid + (int64_t)BIN_PER * NT; k < e; k += NT) {
    uint64_t h;
    T v;
    entry_at(R, pack, w, k, &h, &v);
    insert(h, v, 0, ~0ull);
  }
  __syncthreads();
  int64_t terms = 0;
  if (!s_over) {
    terms = emit(0, false);
  } else {
    // More distinct codes than slots: the bin again, one hash interval at a
    // time, halving an interval whose codes overflow the table.
    for (int i = tid; i < SLOTS; i += NT) {
      keys[i] = 0;
      vals[i] = T(0);
    }
    uint64_t mn = ~0ull, mx = 0;
    for (int64_t k = s + tid; k < e; k += NT) {
      uint64_t h;
      T v;
      entry_at(R, pack, w, k, &h, &v);
      mn = h < mn ? h : mn;
      mx = h > mx ? h : mx;
    }
    mn = block_reduce<NT>(mn, [](uint64_t x, uint64_t y) { return x < y ? x : y; });
    mx = block_reduce<NT>(mx, [](uint64_t x, uint64_t y) { return x > y ? x : y; });
    if (tid == 0) {
      s_lo[0] = mn;
      s_hi[0] = mx;
      s_sp = 1;
    }
    __syncthreads();
    while (s_sp > 0) {
      const uint64_t ilo = s_lo[s_sp - 1], ihi = s_hi[s_sp - 1];
      __syncthreads();
      if (tid == 0) {
        s_over = 0;
        --s_sp;
      }
      __syncthreads();
      for (int64_t k = s + tid; k < e; k += NT) {
        uint64_t h;
        T v;
        entry_at(R, pack, w, k, &h, &v);
        insert(h, v, ilo, ihi);
      }
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
        for (int i = tid; i < SLOTS; i += NT) {
          keys[i] = 0;
          vals[i] = T(0);
        }
        __syncthreads();
      } else {
        terms += emit(terms, true);
      }
    }
  }
  if (tid == 0) R.bin_terms[b] = terms;
  if (R.stats) {
    for (int off = 32; off > 0; off >>= 1) {
      ins += __shfl_xor(ins, off);
      extra += __shfl_xor(extra, off);
    }
    if (lane == 0) {
      atomicAdd(&R.stats[0], (unsigned long long)ins);
      atomicAdd(&R.stats[1], (unsigned long long)extra);
    }
  }
}

// ------------------------------------------------------------ contiguous result
// Each bin's terms fill the first of its entry slots.  With N result terms,
// the terms at N or beyond move into the empty slots below N: the k-th such
// term (in bin order) into the k-th empty slot (in bin order).
// One workgroup per range: the range's result terms (into rhole, as scratch).
__global__ void __launch_bounds__(SMALL_BLOCK) k_rg_fix0(RangeArgs R) {
  if (!R.meta->reserve) return;
  const int64_t r = blockIdx.x;
  int64_t t = 0;
  for (int64_t b = R.rbin0[r] + threadIdx.x; b < R.rbin0[r + 1]; b += SMALL_BLOCK)
    t += R.bin_terms[b];
  t = block_reduce<SMALL_BLOCK>(t, [](int64_t x, int64_t y) { return x + y; });
  if (threadIdx.x == 0) R.rhole[r] = t;
}

// One workgroup: the number of result terms N.
__global__ void __launch_bounds__(1024) k_rg_fixn(RangeArgs R) {
  if (!R.meta->reserve) return;
  int64_t t = 0;
  for (int64_t r = threadIdx.x; r < R.nr; r += 1024) t += R.rhole[r];
  t = block_reduce<1024>(t, [](int64_t x, int64_t y) { return x + y; });
  if (threadIdx.x == 0) R.meta->out_count = t;
}

// One workgroup per range: each bin's empty slots below N and terms at N or
// beyond, as prefix sums within the range, and the range's totals.
__global__ void __launch_bounds__(SMALL_BLOCK) k_rg_fix1(RangeArgs R) {
  if (!R.meta->reserve) return;
  const int64_t r = blockIdx.x;
  const int64_t N = R.meta->out_count;
  const int64_t b0 = R.rbin0[r], nbin = R.rbin0[r + 1] - b0;
  const int64_t per = (nbin + SMALL_BLOCK - 1) / SMALL_BLOCK;
  const int64_t k0 = min(nbin, (int64_t)threadIdx.x * per), k1 = min(nbin, k0 + per);
  const auto hole = [&](int64_t b) -> int64_t {
    const int64_t S = R.bin_start[b], P = R.bin_start[b + 1] - S, T_ = R.bin_terms[b];
    return S + T_ < N ? min(S + P, N) - (S + T_) : 0;
  };
  const auto above = [&](int64_t b) -> int64_t {
    const int64_t S = R.bin_start[b], T_ = R.bin_terms[b];
    return S + T_ > N ? S + T_ - max(S, N) : 0;
  };
  int64_t hl = 0, al = 0;
  for (int64_t k = k0; k < k1; ++k) {
    hl += hole(b0 + k);
    al += above(b0 + k);
  }
  __shared__ int64_t s_ws[SMALL_BLOCK / 64 + 1];
  int64_t htot, atot;
  int64_t hrun = block_scan<SMALL_BLOCK, int64_t>(hl, s_ws, &htot);
  int64_t arun = block_scan<SMALL_BLOCK, int64_t>(al, s_ws, &atot);
  for (int64_t k = k0; k < k1; ++k) {
    R.bhole[b0 + k] = hrun;
    R.babove[b0 + k] = arun;
    hrun += hole(b0 + k);
    arun += above(b0 + k);
  }
  if (threadIdx.x == 0) {
    R.rhole[r] = htot;
    R.rabove[r] = atot;
  }
}

// One workgroup: prefix sums of the ranges' totals (rhole[nr], rabove[nr]:
// all of them, which must agree).
__global__ void __launch_bounds__(1024) k_rg_fix2(RangeArgs R) {
  if (!R.meta->reserve) return;
  const int64_t nr = R.nr;
  const int64_t h = block_scan_runs<1024, int64_t>(R.rhole, nr);
  const int64_t a = block_scan_runs<1024, int64_t>(R.rabove, nr);
  if (threadIdx.x == 0) {
    R.rhole[nr] = h;
    R.rabove[nr] = a;
    if (h != a) atomicOr(&R.meta->err, 1u);   // cannot happen: reported as a device error
  }
}

// The moves, spread over the whole grid: the source and destination of the
// k-th move are found by bisection over the ranges, then over the bins of
// one range.
template <typename T>
__global__ void __launch_bounds__(SMALL_BLOCK) k_rg_fixmove(RangeArgs R) {
  if (!R.meta->reserve) return;
  const int64_t N = R.meta->out_count;
  const int64_t nr = R.nr;
  const int64_t moves = R.rabove[nr];
  const int nx = R.dec.nx;
  T* out_c = static_cast<T*>(R.out_c);
  // the last index g in [a, z) with pre[g] <= k, for pre ascending and pre[a] <= k
  const auto last_le = [](const int64_t* pre, int64_t a, int64_t z, int64_t k) -> int64_t {
    while (z - a > 1) {
      const int64_t m = (a + z) / 2;
      if (pre[m] <= k) a = m;
      else z = m;
    }
    return a;
  };
  for (int64_t k = (int64_t)blockIdx.x * SMALL_BLOCK + threadIdx.x; k < moves;
       k += (int64_t)gridDim.x * SMALL_BLOCK) {
    const int64_t rs = last_le(R.rabove, 0, nr + 1, k);
    const int64_t ks = k - R.rabove[rs];
    const int64_t bsrc = last_le(R.babove, R.rbin0[rs], R.rbin0[rs + 1], ks);
    const int64_t p = max(R.bin_start[bsrc], N) + (ks - R.babove[bsrc]);
    const int64_t rd = last_le(R.rhole, 0, nr + 1, k);
    const int64_t kd = k - R.rhole[rd];
    const int64_t bdst = last_le(R.bhole, R.rbin0[rd], R.rbin0[rd + 1], kd);
    const int64_t q = R.bin_start[bdst] + R.bin_terms[bdst] + (kd - R.bhole[bdst]);
    if (R.out_x) {
      for (int v = 0; v < nx; ++v) R.out_x[q * nx + v] = R.out_x[p * nx + v];
    } else {
      R.out_k[q] = R.out_k[p];
    }
    out_c[q] = out_c[p];
  }
}

template <typename T, int LOG>
void launch_bins(const RangeArgs& R, hipStream_t s) {
  hipLaunchKernelGGL((k_rg_bins<T, LOG>), dim3((unsigned)R.nbins_max), dim3((1 << LOG) / BIN_PER),
                     0, s, R);
}

template <typename T>
hipError_t launch_typed(const RangeArgs& R, hipStream_t s) {
  const dim3 grid((unsigned)R.nr, (unsigned)R.nsplit);
  if (R.ev0) (void)hipEventRecord(R.ev0, s);
  hipLaunchKernelGGL(k_rg_bsort<T>, dim3(1), dim3(SORT_BLOCK), (size_t)R.nbkB * 4, s, R);
  if (R.nb > 0)
    hipLaunchKernelGGL(k_rg_bplace, dim3((unsigned)((R.nb + SMALL_BLOCK - 1) / SMALL_BLOCK)),
                       dim3(SMALL_BLOCK), 0, s, R);
  hipLaunchKernelGGL(k_rg_count0<T>, grid, dim3(SMALL_BLOCK), 0, s, R);
  hipLaunchKernelGGL(k_rg_plan<T>, dim3(1), dim3(1024), 0, s, R);
  const dim3 units((unsigned)(R.nr * R.nsplit));   // walking every (range, split) unit
  hipLaunchKernelGGL(k_rg_count1<T>, units, dim3(RG_BLOCK), 0, s, R);
  hipLaunchKernelGGL(k_rg_scan1, dim3((unsigned)R.nr), dim3(1024), 0, s, R);
  hipLaunchKernelGGL(k_rg_scan2, dim3(1), dim3(1024), 0, s, R);
  hipLaunchKernelGGL(k_rg_scatter<T>, units, dim3(RG_BLOCK), 0, s, R);
  if (R.bin_log >= 13) launch_bins<T, 13>(R, s);
  else if (R.bin_log == 12) launch_bins<T, 12>(R, s);
  else launch_bins<T, 11>(R, s);
  hipLaunchKernelGGL(k_rg_fix0, dim3((unsigned)R.nr), dim3(SMALL_BLOCK), 0, s, R);
  hipLaunchKernelGGL(k_rg_fixn, dim3(1), dim3(1024), 0, s, R);
  hipLaunchKernelGGL(k_rg_fix1, dim3((unsigned)R.nr), dim3(SMALL_BLOCK), 0, s, R);
  hipLaunchKernelGGL(k_rg_fix2, dim3(1), dim3(1024), 0, s, R);
  hipLaunchKernelGGL(k_rg_fixmove<T>, dim3(1024), dim3(SMALL_BLOCK), 0, s, R);
  if (R.ev1) (void)hipEventRecord(R.ev1, s);
  return hipGetLastError();
}

}  // namespace

hipError_t range_setup() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rg_bsort<int64_t>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(DENSE_MAX_BUCKETS * 4));
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rg_bsort<double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(DENSE_MAX_BUCKETS * 4));
  if (e == hipSuccess) done = true;
  return e;
}

hipError_t launch_range(const RangeArgs& R, kp_dtype dt, hipStream_t s) {
  if (R.na == 0 || R.nb == 0 || R.nr == 0) return hipSuccess;
  hipError_t e = range_setup();
  if (e != hipSuccess) return e;
  return dt == KP_F64 ? launch_typed<double>(R, s) : launch_typed<int64_t>(R, s);
}

}  // namespace kp
