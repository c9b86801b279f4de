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
// Work decomposition.  Factor B is cut into tiles of 16 consecutive sorted
// terms, one per lane of a 16-lane DPP row.  For a window [L, L+S) and a tile
// with codes in [bmin, bmax], the rows of A that can land in the window have
// codes in [L - bmax, L + S - bmin): a run of A's buckets, read off the bucket
// start table in O(1).  Rows whose bucket lies inside [L - bmin, L + S - bmax)
// land for every lane ("core" rows); the others ("edge" rows) need a range
// test.  The rows of every (window, tile) pair are cut into work items of at
// most 64 rows, edge and core rows in separate items.  A wavefront handles an
// item as 16 instructions of 64 pairs: lane 16g + v pairs term v of the tile
// with row 16g + u of the item in instruction u, the row's code and
// coefficient being broadcast inside each 16-lane row by DPP row_newbcast:u,
// which folds into the add and the 24-bit multiplies.  The four rows of an
// instruction lie 16 rows apart, so their slots rarely coincide.  An item of
// n < 64 rows (the last of a range) takes only R = 4 ceil(n / 16)
// instructions, lane 16g + u then holding row R g + u: at most 15 idle rows
// per range instead of 63.  The edge test is one
// unsigned min that sends an out-of-window pair to a per-lane discard slot.
//
// Launches (one stream):
//  1. prep    -- two workgroups, one per factor: bucket histogram of the codes
//                in LDS (buckets of 2^shift codes) with each term's rank in
//                its bucket, scan to bucket starts, coefficient-range flags.
//  2. scatter -- one thread per term: writes the bucket-sorted packed
//                {code, low coefficient word} arrays and each tile's code
//                min/max (tiles of 16 consecutive sorted terms of B).
//  3. count   -- one workgroup per window: row ranges of every tile (kept),
//                the window's rows and items; the last workgroup to finish
//                lays out items over all windows and cuts the rows into
//                equal tasks.
//  4. items   -- one workgroup per window: writes the window's work items in
//                (tile, row) order, spread evenly over the threads, and the
//                first item (and window) of every task that starts in it.
//  5. mul     -- one workgroup per task: a task is a run of items of equal
//                rows that may cross windows; for each window it meets it
//                clears the LDS window, wavefronts take the items round-robin
//                with the next item's rows and terms loaded while the current
//                one is accumulated, and the window is flushed: compacted
//                straight from LDS when the task holds all of it, otherwise
//                added into an HBM accumulator with device-scope atomics.
//  6. combine -- one workgroup per chunk of a window split across tasks:
//                compacts the accumulated chunk.
//  7. scan    -- one workgroup: output offset of every chunk, result count
//                (products of more than COPY_SCAN_MAX chunks only).
//  8. copy    -- one workgroup per chunk: moves the chunk to its offset; for
//                at most COPY_SCAN_MAX chunks it sums the counts before its
//                own and the first workgroup publishes the result count.
//
// 128-bit coefficients (exact int64 products): a window holds half as many
// codes, as two arrays of 64-bit words, the low words of its slots followed
// by their high words (two arrays rather than 16-byte slots, so that both
// kinds of add spread over every LDS bank).  Every pair adds its exact
// product with two 64-bit LDS atomics: the add on the low word returns the
// word's previous value, which gives the carry out of that add, and the high
// word then receives the product's high word plus the carry.  The sum of a
// slot is exact in any order of the adds, because each carry out of the low
// word is counted once, by the add that produced it.
#include <algorithm>
#include <climits>
#include <type_traits>
#include <utility>

#include "kp_internal.h"

namespace kp {

namespace {

constexpr int PREP_BLOCK = 1024;
constexpr int PLAN_BLOCK = 1024;
constexpr int64_t ITEMS_LDS_BYTES = 144 * 1024;   // tile rows and item map of the items kernel
constexpr int PREP_UNROLL = 16;   // one round of loads for factors of up to 16384 terms
// Byte offsets that can never fall inside a window (codes are below 2^27, so
// a window offset times 8 stays within +-2^30): a missing row of A, and a
// missing term of B in the last tile.  Their sum is also out of range.
constexpr uint32_t ROW_SENTINEL = 0x80000000u;
constexpr uint32_t LANE_SENTINEL = 0x40000000u;

// Per-window planning records, stored as five arrays of nwin + 1 entries.
enum { W_ITEMS = 0, W_COST = 1, W_SPLIT = 2, W_IBASE = 3, W_CBASE = 4 };
// Task costs count blocks of four instructions: 4 for an item of 64 rows,
// ceil(n / 16) for a shorter one (its instructions, over four).  Equal item
// counts per task left the busiest task 11 % above the median.
// Cost of a window to a task beyond its items (clearing the LDS window, the
// first loads and the flush): that of 64 full items.
constexpr int64_t WINDOW_COST = 64 * 4;

__device__ __forceinline__ int64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// DPP move of a 64-bit value; lanes without a source keep `fill`.
template <int CTRL>
__device__ __forceinline__ int64_t dpp64(int64_t v, int64_t fill) {
  const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)fill, (int)(uint32_t)v, CTRL, 0xF,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)((uint64_t)fill >> 32),
                                             (int)(uint32_t)((uint64_t)v >> 32), CTRL, 0xF, 0xF,
                                             false);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Inclusive wavefront scan without LDS traffic: Hillis-Steele steps inside
// each 16-lane row (DPP row_shr:1,2,4,8), then the row totals by readlane.
// All 64 lanes must be active.
template <bool MAX>
__device__ __forceinline__ int64_t wave_inclusive(int64_t v, int64_t ident) {
  auto op = [](int64_t a, int64_t b) { return MAX ? (a > b ? a : b) : a + b; };
  v = op(v, dpp64<0x111>(v, ident));
  v = op(v, dpp64<0x112>(v, ident));
  v = op(v, dpp64<0x114>(v, ident));
  v = op(v, dpp64<0x118>(v, ident));
  const int row = (threadIdx.x & 63) >> 4;
  const int64_t r0 = readlane64(v, 15), r1 = readlane64(v, 31), r2 = readlane64(v, 47);
  v = op(v, row >= 1 ? r0 : ident);
  v = op(v, row >= 2 ? r1 : ident);
  v = op(v, row >= 3 ? r2 : ident);
  return v;
}

// Block-wide exclusive scan of one int64 per thread; returns the exclusive
// prefix and writes the block total.  Two barriers.
template <int BS>
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* s_wave, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t inc = wave_inclusive<false>(v, 0);
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

// Block-wide exclusive max-scan (identity `lowest`); writes the block maximum.
template <int BS>
__device__ __forceinline__ int64_t block_exclusive_max(int64_t v, int64_t lowest, int64_t* s_wave,
                                                       int64_t* all_max) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t inc = wave_inclusive<true>(v, lowest);
  int64_t ex = __shfl_up(inc, 1);
  if (lane == 0) ex = lowest;
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  int64_t before = lowest, all = lowest;
#pragma unroll
  for (int w = 0; w < BS / 64; ++w) {
    int64_t x = s_wave[w];
    if (w < wave) before = max(before, x);
    all = max(all, x);
  }
  __syncthreads();
  *all_max = all;
  return max(before, ex);
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
  uint64_t* out_pk;       // {code, low coefficient word}
  uint64_t* out_coef;     // coefficient bits
  int32_t* rank;          // [n] rank of each term in its bucket
  int32_t* bstart;        // [nbk + 1] first sorted position of each bucket
  int64_t* tmin;          // [ceil(n/16)] (factor B only, else null)
  int64_t* tmax;
  int64_t* zero;          // array cleared by this workgroup (chunk counts), may be null
  int64_t nzero;
  const int32_t* deg_in;  // optional truncation table (slack of A / degree of B), input order
  int32_t* deg_out;       // the same in bucket-sorted order
};
struct PrepArgs {
  PrepSeg seg[2];
  Meta* meta;
  int is_i64;
};

// Bucket of a code (codes outside the factor's box are flagged by the caller
// and clamped into the first or last bucket).
__device__ __forceinline__ int64_t bucket_of(int64_t k, int shift, int64_t maxb) {
  const int64_t b = k >> shift;
  return k < 0 ? 0 : (b > maxb ? maxb : b);
}

__global__ void __launch_bounds__(PREP_BLOCK) k_dense_prep(PrepArgs args) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int32_t* hist = reinterpret_cast<int32_t*>(smem_raw);
  __shared__ int64_t s_wave[PREP_BLOCK / 64];
  __shared__ uint32_t s_flags[PREP_BLOCK / 64];
  __shared__ uint32_t s_err[PREP_BLOCK / 64];
  constexpr int NW = PREP_BLOCK / 64;
  const int which = blockIdx.x;
  const PrepSeg sg = args.seg[which];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t nbk = sg.nbk;
  const int64_t maxb = nbk - 1;

  if (which == 0 && tid == 0) {
    args.meta->plan_done = 0;
    args.meta->err = 0;
  }
  for (int64_t b = tid; b < nbk; b += PREP_BLOCK) hist[b] = 0;
  for (int64_t i = tid; i < sg.nzero; i += PREP_BLOCK) sg.zero[i] = 0;
  if (sg.tmin) {
    const int64_t ntiles = (sg.n + DENSE_TILE - 1) / DENSE_TILE;
    for (int64_t t = tid; t < ntiles; t += PREP_BLOCK) {
      sg.tmin[t] = LLONG_MAX;
      sg.tmax[t] = LLONG_MIN;
    }
  }
  __syncthreads();
  uint32_t flags = 7u;   // bit0 fits int32, bit1 fits signed 24 bits, bit2 in [0, 2^16)
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
      if (k < 0 || k > sg.maxcode) err |= ERR_RANGE;   // a code outside the factor's box
      sg.rank[i] = atomicAdd(&hist[bucket_of(k, sg.shift, maxb)], 1);
      const int64_t c = cc[u];
      if (c < INT_MIN || c > INT_MAX) flags &= ~1u;
      if (c < -(1 << 23) || c >= (1 << 23)) flags &= ~2u;
      if (c < 0 || c >= (1 << 16)) flags &= ~4u;
    }
  }
  __syncthreads();
  // Exclusive scan of the histogram: thread t owns the contiguous buckets
  // [t per, (t + 1) per), read four at a time (loads in flight) and summed;
  // the sums are scanned across the workgroup, each thread writes its
  // buckets' starts back into LDS, and the workgroup copies them out with
  // consecutive lanes on consecutive buckets.
  const int64_t per = (nbk + PREP_BLOCK - 1) / PREP_BLOCK;
  const int64_t r0 = min(nbk, (int64_t)tid * per), r1 = min(nbk, r0 + per);
  int64_t part = 0;
  for (int64_t b = r0; b < r1; b += 4) {
    int32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = b + u < r1 ? hist[b + u] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) part += v[u];
  }
  int64_t all;
  int64_t run = block_exclusive_scan<PREP_BLOCK>(part, s_wave, &all);
  for (int64_t b = r0; b < r1; b += 4) {
    int32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = b + u < r1 ? hist[b + u] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (b + u < r1) {
        hist[b + u] = (int32_t)run;
        run += v[u];
      }
  }
  __syncthreads();
  for (int64_t b = tid; b < nbk; b += PREP_BLOCK) sg.bstart[b] = hist[b];
  if (tid == 0) sg.bstart[nbk] = (int32_t)sg.n;
  if (!args.is_i64) flags = 0;
  const uint32_t wf = wave_and(flags), we = wave_or(err);
  if (lane == 0) {
    s_flags[wave] = wf;
    s_err[wave] = we;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t f = 7u, e = 0;
    for (int w = 0; w < NW; ++w) {
      f &= s_flags[w];
      e |= s_err[w];
    }
    args.meta->seg_flags[which] = f;
    args.meta->seg_err[which] = e;
  }
}

constexpr int SCATTER_BLOCK = 256;

// Writes every term at its bucket-sorted position; for factor B also the
// code range of each tile of 16 consecutive sorted terms.
__global__ void __launch_bounds__(SCATTER_BLOCK) k_dense_scatter(PrepArgs args, int64_t blocksA) {
  const bool isB = blockIdx.x >= blocksA;
  const PrepSeg& sg = isB ? args.seg[1] : args.seg[0];
  const int64_t i = (int64_t)(isB ? blockIdx.x - blocksA : blockIdx.x) * SCATTER_BLOCK + threadIdx.x;
  if (i >= sg.n) return;
  const int64_t k = sg.keys[i], c = sg.coef[i];
  const int64_t pos = sg.bstart[bucket_of(k, sg.shift, sg.nbk - 1)] + sg.rank[i];
  sg.out_pk[pos] = (uint64_t)(uint32_t)k | ((uint64_t)(uint32_t)c << 32);
  sg.out_coef[pos] = (uint64_t)c;
  if (sg.deg_out) sg.deg_out[pos] = sg.deg_in[i];
  if (isB) {
    const int64_t t = pos / DENSE_TILE, code = (int64_t)(uint32_t)k;
    __hip_atomic_fetch_min(&sg.tmin[t], code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_max(&sg.tmax[t], code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------------ plan
struct PlanArgs {
  int64_t S, nwin, ntiles, nkeys, nb, target, min_work, items_cap;
  int64_t items_lds;     // dynamic LDS bytes of the items kernel
  int accumulate;        // the HBM accumulator was cleared beforehand
  const int32_t* bstart;
  int shiftA;
  int64_t nbkA;
  const int64_t* tmin;
  const int64_t* tmax;
  int64_t* win;          // [5 * (nwin + 1)]
  int4* recs;            // [nwin * ntiles] rows of every (window, tile)
  uint64_t* items;
  int32_t* task_w;
  int32_t* task_begin;
  int64_t* dense;        // [nwin * S * cw] accumulator of windows split across tasks
  Meta* meta;
  int cw;                // words per coefficient (1, or 2 for 128-bit)
};

// Rows of A visited by tile t in the window [L, L + Sw): edge rows [i0, c0),
// core rows [c0, c1) (every lane lands), edge rows [c1, i1).
struct TileRows {
  int64_t i0, c0, c1, i1;
};

__device__ __forceinline__ TileRows tile_rows(const PlanArgs& P, int64_t L, int64_t Sw, int64_t t) {
  TileRows g{0, 0, 0, 0};
  if (t >= P.ntiles) return g;
  const int64_t lo = P.tmin[t], hi = P.tmax[t];
  // the core-row bounds depend only on the tile's codes: their loads go out
  // with those of the row range (one round of latency instead of two)
  const bool full = (t + 1) * DENSE_TILE <= P.nb;
  const int64_t clo = max(L - lo, (int64_t)0), chi = L + Sw - hi;
  const int64_t bw = (int64_t)1 << P.shiftA;
  const int64_t b0 = min((clo + bw - 1) >> P.shiftA, P.nbkA);
  const int64_t b1 = max((int64_t)0, min(chi >> P.shiftA, P.nbkA));
  const bool core = full && chi > clo && b1 > b0;
  const int64_t s0 = core ? P.bstart[b0] : 0, s1 = core ? P.bstart[b1] : 0;
  rows_for(P.bstart, P.shiftA, P.nbkA, L - hi, L + Sw - lo, &g.i0, &g.i1);
  g.c0 = g.c1 = g.i0;
  if (core && g.i1 > g.i0) {
    g.c0 = min(g.i1, max(g.i0, s0));
    g.c1 = min(g.i1, max(g.c0, s1));
  }
  return g;
}

__device__ __forceinline__ int64_t chunks(int64_t n) {
  return (n + DENSE_ITEM_ROWS - 1) / DENSE_ITEM_ROWS;
}

__device__ __forceinline__ uint64_t pack_item(int64_t r0, int64_t t, int64_t n, bool core) {
  const uint32_t hi = (uint32_t)t | ((uint32_t)(n - 1) << 25) | (core ? 0x80000000u : 0u);
  return (uint64_t)(uint32_t)r0 | ((uint64_t)hi << 32);
}

// Tiles [t0, t1) of this thread: a contiguous run, so that one block scan
// orders all of a window's items.
__device__ __forceinline__ void thread_tiles(int64_t ntiles, int64_t* t0, int64_t* t1) {
  const int64_t m = (ntiles + PLAN_BLOCK - 1) / PLAN_BLOCK;
  *t0 = min(ntiles, (int64_t)threadIdx.x * m);
  *t1 = min(ntiles, *t0 + m);
}

__device__ __forceinline__ int64_t items_of(const int4& r) {
  return chunks(r.y - r.x) + chunks(r.z - r.y) + chunks(r.w - r.z);
}

// Cost of a run of n rows cut into items (every item but the last is full),
// of a tile's three runs, of an item of n rows, and of the items of a tile
// before its item k.
__device__ __forceinline__ int64_t run_cost(int64_t n) {
  return 4 * (n / DENSE_ITEM_ROWS) + (n % DENSE_ITEM_ROWS + 15) / 16;
}
__device__ __forceinline__ int64_t cost_of(const int4& r) {
  return run_cost(r.y - r.x) + run_cost(r.z - r.y) + run_cost(r.w - r.z);
}
__device__ __forceinline__ int64_t item_cost(int64_t n) { return (n + 15) / 16; }
// Exclusive block scan of each thread's items and cost.  When every thread
// holds fewer than 2^21 items and a cost below 2^22, the totals stay below
// 2^31 and 2^32, and items (high 31 bits) and cost (low 33 bits) are scanned
// as one value; otherwise in two scans.
constexpr int COST_BITS = 33;
__device__ __forceinline__ void scan_items_cost(int64_t nit, int64_t cost, int64_t* s_wave,
                                                int64_t* q, int64_t* qc, int64_t* tot_items,
                                                int64_t* tot_cost) {
  if (!__syncthreads_or(nit >= ((int64_t)1 << 21) || cost >= ((int64_t)1 << 22))) {
    int64_t tot;
    const uint64_t v = (uint64_t)block_exclusive_scan<PLAN_BLOCK>(
        (int64_t)(((uint64_t)nit << COST_BITS) | (uint64_t)cost), s_wave, &tot);
    const uint64_t mask = ((uint64_t)1 << COST_BITS) - 1;
    *q = (int64_t)(v >> COST_BITS);
    *qc = (int64_t)(v & mask);
    *tot_items = (int64_t)((uint64_t)tot >> COST_BITS);
    *tot_cost = (int64_t)((uint64_t)tot & mask);
  } else {
    *q = block_exclusive_scan<PLAN_BLOCK>(nit, s_wave, tot_items);
    *qc = block_exclusive_scan<PLAN_BLOCK>(cost, s_wave, tot_cost);
  }
}


// Item k of a tile with rows {i0, c0, c1, i1}: first row, rows, core flag,
// and the cost of the tile's items before it (every item of a run but the
// last is full, cost 4).
__device__ __forceinline__ void item_rows(const int4& r, int64_t k, int64_t* r0, int64_t* n,
                                          bool* core, int64_t* before) {
  const int64_t e1 = chunks(r.y - r.x), ec = chunks(r.z - r.y);
  int64_t hi;
  if (k < e1) {
    *r0 = r.x + k * DENSE_ITEM_ROWS;
    hi = r.y;
    *core = false;
    *before = 4 * k;
  } else if (k < e1 + ec) {
    *r0 = r.y + (k - e1) * DENSE_ITEM_ROWS;
    hi = r.z;
    *core = true;
    *before = run_cost(r.y - r.x) + 4 * (k - e1);
  } else {
    *r0 = r.z + (k - e1 - ec) * DENSE_ITEM_ROWS;
    hi = r.w;
    *core = false;
    *before = run_cost(r.y - r.x) + run_cost(r.z - r.y) + 4 * (k - e1 - ec);
  }
  *n = min(DENSE_ITEM_ROWS, hi - *r0);
  *core = *core && *n == DENSE_ITEM_ROWS;
}

// Products of at most this many windows lay out their tasks in the items
// kernel (every workgroup sums the records of the windows before its own);
// larger ones in the last workgroup of the count kernel.
constexpr int64_t LAYOUT_IN_ITEMS_MAX = 4096;

// Workgroup-wide sums of four values per thread (every thread gets them):
// DPP wavefront sums, one barrier.  s_red is written once per kernel.
__device__ __forceinline__ void block_sum4(int64_t (&v)[4], int64_t* s_red) {
  constexpr int NW = PLAN_BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = readlane64(wave_inclusive<false>(v[k], 0), 63);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) s_red[k * NW + wave] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int64_t t = 0;
    for (int u = 0; u < NW; ++u) t += s_red[k * NW + u];
    v[k] = t;
  }
}

// Task size from the total cost: tasks of equal cost T (more than one
// window's overhead plus an item's); task p starts at the item whose cost
// interval holds p * T.
__device__ __forceinline__ void task_shape(const PlanArgs& P, int64_t all_cost, int64_t* T,
                                           int64_t* nt) {
  int64_t t = (all_cost + P.target - 1) / P.target;
  if (t < WINDOW_COST + 4) t = WINDOW_COST + 4;
  *T = t;
  *nt = all_cost > 0 ? (all_cost + t - 1) / t : 0;
}

__global__ void __launch_bounds__(PLAN_BLOCK) k_dense_count(PlanArgs P) {
  __shared__ int64_t s_wave[PLAN_BLOCK / 64];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int64_t L = w * P.S;
  const int64_t Sw = min(P.S, P.nkeys - L);
  const int64_t W1 = P.nwin + 1;
  int4* rec = P.recs + w * P.ntiles;
  int64_t t0, t1;
  thread_tiles(P.ntiles, &t0, &t1);
  int64_t nit = 0, cost = 0;
  constexpr int BATCH = 4;   // tiles whose loads are issued together
  for (int64_t t = t0; t < t1; t += BATCH) {
    TileRows g[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) g[u] = tile_rows(P, L, Sw, min(t + u, t1 - 1));
#pragma unroll
    for (int u = 0; u < BATCH; ++u)
      if (t + u < t1) {
        const int4 r = make_int4((int)g[u].i0, (int)g[u].c0, (int)g[u].c1, (int)g[u].i1);
        rec[t + u] = r;
        nit += items_of(r);
        cost += cost_of(r);
      }
  }
  int64_t q, qc, tot_items, tot_cost;
  scan_items_cost(nit, cost, s_wave, &q, &qc, &tot_items, &tot_cost);
  if (P.nwin <= LAYOUT_IN_ITEMS_MAX) {   // the items kernel lays out the tasks
    if (tid == 0) {
      P.win[W_ITEMS * W1 + w] = tot_items;
      P.win[W_COST * W1 + w] = tot_cost;
    }
    return;
  }
  if (tid == 0) {
    P.win[W_ITEMS * W1 + w] = tot_items;
    P.win[W_COST * W1 + w] = tot_cost;
    __threadfence();
    s_last = atomicAdd(&P.meta->plan_done, 1u) == (uint32_t)(P.nwin - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // last workgroup: item and row offsets of every window, equal tasks
  auto ld = [&](int k, int64_t u) {
    return __hip_atomic_load(&P.win[k * W1 + u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  const int64_t per = (P.nwin + PLAN_BLOCK - 1) / PLAN_BLOCK;
  const int64_t w0 = min(P.nwin, tid * per), w1 = min(w0 + per, P.nwin);
  // each thread's windows, read once (kept in registers for up to 4)
  constexpr int KEEP = 4;
  int64_t kept[KEEP], kept_c[KEEP];
  int64_t li = 0, lc = 0;   // items, and cost: the items' plus WINDOW_COST when any
  for (int64_t u = w0; u < w1; ++u) {
    const int64_t it = ld(W_ITEMS, u), ct = ld(W_COST, u);
    if (u - w0 < KEEP) {
      kept[u - w0] = it;
      kept_c[u - w0] = ct;
    }
    li += it;
    lc += it > 0 ? ct + WINDOW_COST : 0;
  }
  int64_t ibase, cbase, all_items, all_cost;
  scan_items_cost(li, lc, s_wave, &ibase, &cbase, &all_items, &all_cost);
  for (int64_t u = w0; u < w1; ++u) {
    const int64_t it = u - w0 < KEEP ? kept[u - w0] : ld(W_ITEMS, u);
    const int64_t ct = u - w0 < KEEP ? kept_c[u - w0] : ld(W_COST, u);
    P.win[W_IBASE * W1 + u] = ibase;
    P.win[W_CBASE * W1 + u] = cbase;
    ibase += it;
    cbase += it > 0 ? ct + WINDOW_COST : 0;
  }
  // No work after a factor code outside its box (reported by the scan
  // kernel), or past the planned item bound (which cannot happen).
  const uint32_t bad = P.meta->seg_err[0] | P.meta->seg_err[1];
  if (tid == 0) {
    P.win[W_IBASE * W1 + P.nwin] = all_items;
    P.win[W_CBASE * W1 + P.nwin] = all_cost;
    int64_t T, nt;
    task_shape(P, all_cost, &T, &nt);
    if (bad || all_items > P.items_cap) {
      P.meta->err |= bad ? bad : ERR_CAPACITY;
      nt = 0;
    }
    P.meta->task_rows = T;
    P.meta->ntasks = nt;
    P.task_begin[nt] = (int32_t)all_items;
  }
}

// Item k of window w: its descriptor, and the first item (and window) of the
// task that starts at it, if any.  Item k covers the cost interval
// [cb + WINDOW_COST + c, + item_cost(n)), c the cost of the window's items
// before it (the first item also covers the window's overhead
// [cb, cb + WINDOW_COST)); task p starts at the item whose interval holds
// p * T.
__device__ __forceinline__ void put_item(const PlanArgs& P, int64_t w, int64_t ib, int64_t k,
                                         int64_t cb, int64_t c, int64_t r0, int64_t t, int64_t n,
                                         bool core, int64_t T, double rT, int* s_split) {
  P.items[ib + k] = pack_item(r0, t, n, core);
  const int64_t lo = k == 0 ? cb : cb + WINDOW_COST + c, hi = cb + WINDOW_COST + c + item_cost(n);
  // smallest p with p * T >= lo (the quotient is exact in double below 2^52)
  int64_t p = (int64_t)ceil((double)lo * rT);
  while (p > 0 && (p - 1) * T >= lo) --p;
  while (p * T < lo) ++p;
  if (p * T < hi) {
    P.task_begin[p] = (int32_t)(ib + k);
    P.task_w[p] = (int32_t)w;
    if (k > 0) *s_split = 1;   // a task starts inside the window
  }
}

__global__ void __launch_bounds__(PLAN_BLOCK) k_dense_items(PlanArgs P) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int64_t s_wave[PLAN_BLOCK / 64];
  __shared__ int s_split;
  const int tid = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int64_t W1 = P.nwin + 1;
  const int64_t nit_w = P.win[W_ITEMS * W1 + w];
  if (tid == 0) s_split = 0;
  const int4* rec = P.recs + w * P.ntiles;
  const int64_t nt = P.ntiles;
  // LDS: the window's tile rows, per-tile item and cost prefixes, tile of
  // every item
  int4* s_rec = reinterpret_cast<int4*>(smem_raw);
  int32_t* s_ip = reinterpret_cast<int32_t*>(s_rec + nt);
  int32_t* s_cp = s_ip + nt + 1;
  int32_t* s_of = s_cp + nt + 1;
  const bool in_lds = (size_t)nt * 24 + 8 + (size_t)nit_w * 4 <= (size_t)P.items_lds;
  // the tile rows go to LDS first, so that their loads overlap the layout's
  if (in_lds && nit_w > 0)
    for (int64_t t = tid; t < nt; t += PLAN_BLOCK) s_rec[t] = rec[t];
  const bool layout_here = P.nwin <= LAYOUT_IN_ITEMS_MAX;
  int64_t ib, cb, T, ntasks;
  if (layout_here) {
    // this window's item and cost offsets, and the task size, from the
    // windows' records (the count kernel's last workgroup does this for
    // larger products)
    __shared__ int64_t s_red[4 * (PLAN_BLOCK / 64)];
    // (all loads issued together: the error bits, and both records of the
    // thread's windows)
    const uint32_t bad = P.meta->seg_err[0] | P.meta->seg_err[1];
    int64_t v[4] = {0, 0, 0, 0};   // items before w, cost before w, all items, all cost
    for (int64_t u = tid; u < P.nwin; u += PLAN_BLOCK) {
      const int64_t it = P.win[W_ITEMS * W1 + u], ct = P.win[W_COST * W1 + u];
      const int64_t c = it > 0 ? ct + WINDOW_COST : 0;
      if (u < w) {
        v[0] += it;
        v[1] += c;
      }
      v[2] += it;
      v[3] += c;
    }
    block_sum4(v, s_red);
    ib = v[0];
    cb = v[1];
    task_shape(P, v[3], &T, &ntasks);
    // no work after a factor code outside its box (reported by the scan
    // kernel), or past the planned item bound (which cannot happen)
    if (bad || v[2] > P.items_cap) ntasks = 0;
    if (tid == 0) {
      P.win[W_IBASE * W1 + w] = ib;   // read by the multiply kernel
      if (w == 0) {
        P.win[W_IBASE * W1 + P.nwin] = v[2];
        if (bad || v[2] > P.items_cap) P.meta->err |= bad ? bad : ERR_CAPACITY;
        P.meta->task_rows = T;
        P.meta->ntasks = ntasks;
        P.task_begin[ntasks] = (int32_t)v[2];
      }
    }
  } else {
    ib = P.win[W_IBASE * W1 + w];
    cb = P.win[W_CBASE * W1 + w];
    T = P.meta->task_rows;
    ntasks = P.meta->ntasks;
  }
  if (ntasks == 0 || nit_w == 0) {
    if (tid == 0) P.win[W_SPLIT * W1 + w] = 0;
    return;
  }
  const double rT = 1.0 / (double)T;
  int64_t t0, t1;
  thread_tiles(nt, &t0, &t1);
  if (in_lds) {
    if (!layout_here) __syncthreads();   // the records are in LDS (else the prologue's barrier)
    int64_t nit = 0, ncost = 0;
    for (int64_t t = t0; t < t1; ++t) {
      nit += items_of(s_rec[t]);
      ncost += cost_of(s_rec[t]);
    }
    int64_t q, qc, tq, tqc;
    scan_items_cost(nit, ncost, s_wave, &q, &qc, &tq, &tqc);
    for (int64_t k = tid; k < nit_w; k += PLAN_BLOCK) s_of[k] = -1;
    __syncthreads();
    // each non-empty tile marks its first item; a max-scan over the items
    // then gives every item its tile
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t c = items_of(s_rec[t]);
      s_ip[t] = (int32_t)q;
      s_cp[t] = (int32_t)qc;
      if (c > 0) s_of[q] = (int32_t)t;
      q += c;
      qc += cost_of(s_rec[t]);
    }
    __syncthreads();
    const int64_t per = (nit_w + PLAN_BLOCK - 1) / PLAN_BLOCK;
    const int64_t k0 = min(nit_w, tid * per), k1 = min(nit_w, k0 + per);
    int64_t run = -1;
    for (int64_t k = k0; k < k1; ++k) run = max(run, (int64_t)s_of[k]);
    int64_t all_max;
    run = block_exclusive_max<PLAN_BLOCK>(run, -1, s_wave, &all_max);
    for (int64_t k = k0; k < k1; ++k) {
      run = max(run, (int64_t)s_of[k]);
      s_of[k] = (int32_t)run;
    }
    __syncthreads();
    for (int64_t k = tid; k < nit_w; k += PLAN_BLOCK) {
      const int64_t t = s_of[k];
      const int4 r = s_rec[t];
      int64_t r0, n, before;
      bool core;
      item_rows(r, k - s_ip[t], &r0, &n, &core, &before);
      P.items[ib + k] = pack_item(r0, t, n, core);
    }
    // Tasks that start in this window: task p at the item whose cost
    // interval holds p * T (item 0's interval also covers the window's
    // overhead), found by one thread each by bisection over the items' cost
    // starts.  At most one item in 65 starts a task.
    auto start_of = [&](int64_t k) -> int64_t {   // cost interval start of item k
      if (k == 0) return cb;
      const int64_t t = s_of[k];
      int64_t r0, n, before;
      bool core;
      item_rows(s_rec[t], k - s_ip[t], &r0, &n, &core, &before);
      return cb + WINDOW_COST + s_cp[t] + before;
    };
    const int64_t end = cb + WINDOW_COST + tqc;   // past the window's last item
    for (int64_t p = (cb + T - 1) / T + tid; p * T < end; p += PLAN_BLOCK) {
      const int64_t x = p * T;
      int64_t lo = 0, hi = nit_w - 1;   // largest k with start_of(k) <= x
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (start_of(mid) <= x) lo = mid;
        else hi = mid - 1;
      }
      P.task_begin[p] = (int32_t)(ib + lo);
      P.task_w[p] = (int32_t)w;
      if (lo > 0) s_split = 1;   // a task starts inside the window
    }
  } else {
    // too large for LDS: each thread writes the items of its own tiles
    int64_t nit = 0, ncost = 0;
    for (int64_t t = t0; t < t1; ++t) {
      nit += items_of(rec[t]);
      ncost += cost_of(rec[t]);
    }
    int64_t q, qc, tq, tqc;
    scan_items_cost(nit, ncost, s_wave, &q, &qc, &tq, &tqc);
    for (int64_t t = t0; t < t1; ++t) {
      const int4 r = rec[t];
      const int64_t cnt = items_of(r);
      for (int64_t k = 0; k < cnt; ++k) {
        int64_t r0, n, before;
        bool core;
        item_rows(r, k, &r0, &n, &core, &before);
        put_item(P, w, ib, q + k, cb, qc + before, r0, t, n, core, T, rT, &s_split);
      }
      q += cnt;
      qc += cost_of(r);
    }
  }
  __syncthreads();
  if (s_split && !P.accumulate) {   // tasks of a split window add into the HBM accumulator
    const int64_t L = w * P.S;
    const int64_t Sw = min(P.S, P.nkeys - L);
    int64_t* d = P.dense + L * P.cw;
    for (int64_t i = tid; i < Sw * P.cw; i += PLAN_BLOCK) d[i] = 0;
  }
  if (tid == 0) P.win[W_SPLIT * W1 + w] = s_split;
}

// ------------------------------------------------------------------ multiply
struct MulArgs {
  const Meta* meta;
  const uint64_t* apk;    // A: {code, low coefficient word}
  const uint64_t* ac;     // A: coefficient bits
  const uint64_t* bpk;
  const uint64_t* bc;
  int64_t nb, S, nwin, nkeys;
  const uint64_t* items;
  const int32_t* task_w;
  const int32_t* task_begin;
  const int64_t* win_ibase;   // [nwin + 1] first item of each window
  int accumulate;             // every window adds into the HBM accumulator
  int64_t* dense;
  int64_t* stage_k;
  int64_t* stage_c;
  int64_t* ccount;
  const int32_t* a_sa;   // optional truncation: slack of each row of A (sorted order)
  const int32_t* b_tb;   // and degree of each term of B; a pair is kept iff tb <= sa
};

template <int U>
__device__ __forceinline__ uint32_t bcast16(uint32_t v) {
  // row_newbcast:U -- every lane of a 16-lane row reads lane U of that row
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + U, 0xF, 0xF, false);
}

__device__ __forceinline__ void lds_add(uint32_t addr, int64_t v) {
  typedef __attribute__((address_space(3))) unsigned long long lds_u64;
  __hip_atomic_fetch_add(reinterpret_cast<lds_u64*>((size_t)addr), (unsigned long long)v,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t lds_fetch_add(uint32_t addr, uint64_t v) {
  typedef __attribute__((address_space(3))) unsigned long long lds_u64;
  return __hip_atomic_fetch_add(reinterpret_cast<lds_u64*>((size_t)addr), (unsigned long long)v,
                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(uint32_t addr, double v) {
  typedef __attribute__((address_space(3))) double lds_f64;
  __hip_atomic_fetch_add(reinterpret_cast<lds_f64*>((size_t)addr), v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Coefficient kinds.  MUL: 4 = both factors in [0, 2^16) (one 24-bit
// multiply, the product's high word is zero), 2 = both fit signed 24 bits
// (two 24-bit multiplies), 1 = both fit int32 (one 32x32->64 multiply),
// 0 = general int64 (wraps modulo 2^64), 3 = fp64, 5 = int64 factors with
// exact 128-bit products and sums.
template <typename T, int MUL>
struct Coef {
  uint32_t lo, hi;   // this lane's row of A (broadcast per instruction)
  int32_t bn;        // this lane's term of B, narrow kinds
  T bw;              // this lane's term of B, wide kinds
};

// One instruction of an item: row 4U + g of the item against this lane's term.
// Window byte offsets are relative to the window's LDS base, which is added
// last (it folds into the instruction's offset field).  In a truncated
// product a pair over the degree limit goes to the lane's discard slot, and
// an instruction whose pairs are all over the limit issues no LDS add (a
// wavefront-uniform branch: the broadcasts read other lanes, so the
// execution mask never changes around them).
template <typename T, int MUL, bool EDGE, bool TRUNC, int U>
__device__ __forceinline__ void pair_step(uint32_t a8, uint32_t off8, uint32_t lim, uint32_t base,
                                          const Coef<T, MUL>& c, uint32_t sa, int32_t tb) {
  const bool keep = !TRUNC || (int32_t)bcast16<U>(sa) >= tb;   // within the degree limit
  if (TRUNC && __builtin_amdgcn_ballot_w64(keep) == 0) return;
  uint32_t rel = bcast16<U>(a8) + off8;
  if (EDGE) rel = min(rel, lim);
  if (TRUNC && !keep) rel = lim;
  rel += base;
  T v;
  if constexpr (MUL == 4) {
    const uint32_t x = bcast16<U>(c.lo) & 0xFFFFFFu;
    v = (T)(uint64_t)(x * ((uint32_t)c.bn & 0xFFFFFFu));
  } else if constexpr (MUL == 2) {
    const int32_t x = (int32_t)bcast16<U>(c.lo);
    v = (T)((int64_t)((x << 8) >> 8) * (int64_t)c.bn);
  } else if constexpr (MUL == 1) {
    v = (T)((int64_t)(int32_t)bcast16<U>(c.lo) * (int64_t)c.bn);
  } else if constexpr (MUL == 0) {
    const uint64_t x = ((uint64_t)bcast16<U>(c.hi) << 32) | bcast16<U>(c.lo);
    v = (T)(x * (uint64_t)c.bw);
  } else {
    const uint64_t bits = ((uint64_t)bcast16<U>(c.hi) << 32) | bcast16<U>(c.lo);
    double x;
    __builtin_memcpy(&x, &bits, 8);
    v = (T)(x * (double)c.bw);
  }
  lds_add(rel, v);
}

template <typename T, int MUL, bool EDGE, bool TRUNC, int G, int... U>
__device__ __forceinline__ void item_steps(std::integer_sequence<int, U...>, uint32_t a8,
                                           uint32_t off8, uint32_t lim, uint32_t base,
                                           const Coef<T, MUL>& c, uint32_t sa, int32_t tb) {
  (pair_step<T, MUL, EDGE, TRUNC, G + U>(a8, off8, lim, base, c, sa, tb), ...);
}

// 128-bit slots (MUL 5): the low word's offset is computed as for the other
// kinds (same edge and discard tests); the high word lies hi8 bytes further.
// Issue: the exact product and the low-word add, which returns the old low
// word.
template <bool EDGE, bool TRUNC, int U>
__device__ __forceinline__ void wide_issue(uint32_t a8, uint32_t off8, uint32_t lim, uint32_t base,
                                           uint32_t clo, uint32_t chi, int64_t bw, uint32_t sa,
                                           int32_t tb, uint32_t& addr, uint64_t& plo,
                                           int64_t& phi, uint64_t& old, bool& keep) {
  // wavefront-uniform: false when every pair of the instruction is over the
  // degree limit (no add issued); lanes over the limit use the discard slot
  const bool mine = !TRUNC || (int32_t)bcast16<U>(sa) >= tb;
  keep = !TRUNC || __builtin_amdgcn_ballot_w64(mine) != 0;
  uint32_t rel = bcast16<U>(a8) + off8;
  if (EDGE) rel = min(rel, lim);
  if (TRUNC && !mine) rel = lim;
  addr = rel + base;
  const int64_t x = (int64_t)(((uint64_t)bcast16<U>(chi) << 32) | bcast16<U>(clo));
  plo = (uint64_t)x * (uint64_t)bw;
  phi = __mul64hi(x, bw);
  old = 0;
  if (keep) old = lds_fetch_add(addr, plo);
}

// Finish: the carry out of the low-word add goes into the high word.
__device__ __forceinline__ void wide_finish(uint32_t addr, uint32_t hi8, uint64_t plo,
                                            int64_t phi, uint64_t old, bool keep) {
  const uint64_t carry = old + plo < old ? 1u : 0u;
  if (keep) lds_add(addr + hi8, (int64_t)((uint64_t)phi + carry));
}

// A group of instructions: every low-word add is issued before the first
// returned value is needed, so their latencies overlap.
template <bool EDGE, bool TRUNC, int G, int... U>
__device__ __forceinline__ void wide_group(std::integer_sequence<int, U...>, uint32_t a8,
                                           uint32_t off8, uint32_t lim, uint32_t base,
                                           uint32_t clo, uint32_t chi, int64_t bw, uint32_t sa,
                                           int32_t tb, uint32_t hi8) {
  constexpr int N = sizeof...(U);
  uint32_t addr[N];
  uint64_t plo[N], old[N];
  int64_t phi[N];
  bool keep[N];
  (wide_issue<EDGE, TRUNC, G + U>(a8, off8, lim, base, clo, chi, bw, sa, tb, addr[U], plo[U],
                                  phi[U], old[U], keep[U]),
   ...);
  (wide_finish(addr[U], hi8, plo[U], phi[U], old[U], keep[U]), ...);
}

// R instructions (4, 8, 12 or 16), in groups of up to eight.
template <bool EDGE, bool TRUNC>
__device__ __forceinline__ void wide_steps(uint32_t a8, uint32_t off8, uint32_t lim, uint32_t base,
                                           uint32_t clo, uint32_t chi, int64_t bw, uint32_t sa,
                                           int32_t tb, uint32_t hi8, int R) {
  if (R >= 8)
    wide_group<EDGE, TRUNC, 0>(std::make_integer_sequence<int, 8>{}, a8, off8, lim, base, clo,
                               chi, bw, sa, tb, hi8);
  else
    wide_group<EDGE, TRUNC, 0>(std::make_integer_sequence<int, 4>{}, a8, off8, lim, base, clo,
                               chi, bw, sa, tb, hi8);
  if (R == 16)
    wide_group<EDGE, TRUNC, 8>(std::make_integer_sequence<int, 8>{}, a8, off8, lim, base, clo,
                               chi, bw, sa, tb, hi8);
  else if (R == 12)
    wide_group<EDGE, TRUNC, 8>(std::make_integer_sequence<int, 4>{}, a8, off8, lim, base, clo,
                               chi, bw, sa, tb, hi8);
}

// Instructions of an item of n rows: 4, 8, 12 or 16, so that the four
// 16-lane groups cover the rows in blocks of four instructions (an item of
// 64 rows, every core item, takes all 16).  Lane 16g + u holds row R g + u
// of the item for u < R.
__device__ __forceinline__ int item_instr(int64_t n) { return (int)(((n + 15) >> 4) << 2); }
__device__ __forceinline__ int item_row(int64_t n, int lane) {
  const int R = item_instr(n), u = lane & 15;
  return R * (lane >> 4) + (u < R ? u : R - 1);
}

struct ItemRegs {
  int64_t r0, t, n;
  bool core;
  uint64_t a, b;     // packed rows / terms
  uint64_t ac, bc;   // coefficient words (wide kinds)
  int32_t sa, tb;    // truncation: slack of this lane's row, degree of its term
};

template <bool WIDE, bool TRUNC>
__device__ __forceinline__ void fetch_item(const MulArgs& M, int64_t d, int lane, ItemRegs& x) {
  const uint32_t lo = (uint32_t)d, hi = (uint32_t)((uint64_t)d >> 32);
  x.r0 = (int64_t)lo;
  x.t = (int64_t)(hi & 0x1FFFFFFu);
  x.n = (int64_t)((hi >> 25) & 63u) + 1;
  x.core = (hi >> 31) != 0;
  const int64_t j = min(x.t * DENSE_TILE + (lane & 15), M.nb - 1);
  const int64_t r = x.r0 + min((int64_t)item_row(x.n, lane), x.n - 1);
  x.b = M.bpk[j];
  x.a = M.apk[r];
  if (WIDE) {
    x.bc = M.bc[j];
    x.ac = M.ac[r];
  }
  if (TRUNC) {
    x.sa = M.a_sa[r];
    x.tb = M.b_tb[j];
  }
}

// Smallest value of a 16-lane row, in every lane of the row (rotations).
template <int K>
__device__ __forceinline__ int32_t row_ror(int32_t v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x120 + K, 0xF, 0xF, false);   // row_ror:K
}
__device__ __forceinline__ int32_t row_min16(int32_t v) {
  v = min(v, row_ror<1>(v));
  v = min(v, row_ror<2>(v));
  v = min(v, row_ror<4>(v));
  return min(v, row_ror<8>(v));
}

template <typename T, int MUL, bool TRUNC>
__device__ __forceinline__ void run_item(const ItemRegs& x, int64_t L, uint32_t lim, int lane,
                                         int64_t nb, uint32_t base, uint32_t hi8) {
  // a truncated product skips an item whose every pair is over the degree
  // limit: no row's slack reaches the tile's smallest degree (every lane
  // holds a row of the item and every 16-lane row the tile's terms)
  if (TRUNC && __builtin_amdgcn_ballot_w64(x.sa >= row_min16(x.tb)) == 0) return;
  const bool vb = x.t * DENSE_TILE + (lane & 15) < nb;
  const uint32_t off8 =
      vb ? (uint32_t)(((int32_t)(uint32_t)x.b - (int32_t)L) * 8) : LANE_SENTINEL;
  const int R = item_instr(x.n);   // wavefront-uniform
  const uint32_t a8 = (lane & 15) < R && R * (lane >> 4) + (lane & 15) < x.n
                          ? ((uint32_t)x.a << 3) : ROW_SENTINEL;
  if constexpr (MUL == 5) {
    const uint32_t clo = (uint32_t)x.ac, chi = (uint32_t)(x.ac >> 32);
    const int64_t bw = (int64_t)x.bc;
    if (x.core)
      wide_steps<false, TRUNC>(a8, off8, lim, base, clo, chi, bw, (uint32_t)x.sa, x.tb, hi8, 16);
    else
      wide_steps<true, TRUNC>(a8, off8, lim, base, clo, chi, bw, (uint32_t)x.sa, x.tb, hi8, R);
  } else {
    Coef<T, MUL> c;
    if constexpr (MUL == 1 || MUL == 2 || MUL == 4) {
      c.lo = (uint32_t)(x.a >> 32);
      c.hi = 0;
      c.bn = (int32_t)(uint32_t)(x.b >> 32);
      if constexpr (MUL == 2) c.bn = (c.bn << 8) >> 8;
      c.bw = T(0);
    } else {
      c.lo = (uint32_t)x.ac;
      c.hi = (uint32_t)(x.ac >> 32);
      c.bn = 0;
      __builtin_memcpy(&c.bw, &x.bc, 8);
    }
    if (x.core) {
      item_steps<T, MUL, false, TRUNC, 0>(std::make_integer_sequence<int, 16>{}, a8, off8, lim,
                                          base, c, (uint32_t)x.sa, x.tb);
    } else {   // R instructions, in blocks of four
      constexpr auto q4 = std::make_integer_sequence<int, 4>{};
      item_steps<T, MUL, true, TRUNC, 0>(q4, a8, off8, lim, base, c, (uint32_t)x.sa, x.tb);
      if (R > 4) item_steps<T, MUL, true, TRUNC, 4>(q4, a8, off8, lim, base, c, (uint32_t)x.sa, x.tb);
      if (R > 8) item_steps<T, MUL, true, TRUNC, 8>(q4, a8, off8, lim, base, c, (uint32_t)x.sa, x.tb);
      if (R > 12)
        item_steps<T, MUL, true, TRUNC, 12>(q4, a8, off8, lim, base, c, (uint32_t)x.sa, x.tb);
    }
  }
}

// Items [ib, ie) of the task, wavefront w taking ib + w, ib + w + NW, ...;
// the next item's rows and terms are loaded while the current one runs.
template <typename T, int MUL, int BS, bool TRUNC>
__device__ __forceinline__ void run_items(const MulArgs& M, int64_t ib, int64_t ie, int64_t L,
                                          uint32_t S8, uint32_t base, uint32_t hi8) {
  constexpr int NW = BS / 64;
  constexpr bool WIDE = MUL == 0 || MUL == 3 || MUL == 5;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // out-of-window pairs go to this lane's discard slot (or, within 64 slots
  // past the window, to some discard slot)
  const uint32_t lim = S8 + (uint32_t)lane * 8;
  for (int64_t e0 = ib + wave; e0 < ie; e0 += (int64_t)NW * 64) {
    const int64_t mine = e0 + (int64_t)NW * lane;
    const uint64_t dv = mine < ie ? M.items[mine] : 0;
    const int cnt = (int)min((int64_t)64, (ie - e0 + NW - 1) / NW);
    // two register sets in turn, so that no load result is copied (a copy
    // would wait for the load)
    ItemRegs x0, x1;
    fetch_item<WIDE, TRUNC>(M, readlane64(dv, 0), lane, x0);
    for (int k = 0; k + 1 < cnt; k += 2) {
      fetch_item<WIDE, TRUNC>(M, readlane64(dv, k + 1), lane, x1);
      run_item<T, MUL, TRUNC>(x0, L, lim, lane, M.nb, base, hi8);
      fetch_item<WIDE, TRUNC>(M, readlane64(dv, min(k + 2, cnt - 1)), lane, x0);
      run_item<T, MUL, TRUNC>(x1, L, lim, lane, M.nb, base, hi8);
    }
    if (cnt & 1) run_item<T, MUL, TRUNC>(x0, L, lim, lane, M.nb, base, hi8);
  }
}

__device__ __forceinline__ void global_add(int64_t* p, int64_t v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void global_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void global_add(I128* p, I128 v) {
  unsigned long long* w = reinterpret_cast<unsigned long long*>(p);
  const uint64_t old = atomicAdd(w, (unsigned long long)v.lo);
  const uint64_t carry = old + v.lo < old ? 1u : 0u;
  atomicAdd(w + 1, (unsigned long long)((uint64_t)v.hi + carry));
}

// Slot i of the window: one word, or (128-bit) the low word and the high
// word `hw` words further.
template <typename T>
__device__ __forceinline__ T win_load(const unsigned char* win, int64_t i, int64_t hw) {
  if constexpr (std::is_same<T, I128>::value) {
    const uint64_t* w = reinterpret_cast<const uint64_t*>(win);
    return I128(w[i], (int64_t)w[hw + i]);
  } else {
    return reinterpret_cast<const T*>(win)[i];
  }
}

// Flush of one window piece: compaction straight from LDS when the task
// holds the whole window, else an add of its nonzero slots into HBM.
template <typename T, int BS>
__device__ __forceinline__ void flush_window(const MulArgs& M, const unsigned char* win, int64_t L,
                                             int64_t Sw, int64_t hw, bool whole) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (!whole) {
    T* d = reinterpret_cast<T*>(M.dense) + L;
    for (int64_t i = tid; i < Sw; i += BS) {
      const T v = win_load<T>(win, i, hw);
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
      const T v = i < s1 ? win_load<T>(win, i, hw) : T(0);
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

template <typename T, int BS>
__global__ void __launch_bounds__(BS) k_dense_mul(MulArgs M) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t task = blockIdx.x;
  if (task >= M.meta->ntasks) return;
  const int64_t ib = M.task_begin[task], ie = M.task_begin[task + 1];
  const int tid = threadIdx.x;
  // The kernel has no static LDS, so the window starts at LDS address 0 and
  // the per-pair address arithmetic carries no base.
  constexpr uint32_t base = 0;
  const uint32_t narrow = M.meta->seg_flags[0] & M.meta->seg_flags[1];
  const bool trunc = M.a_sa != nullptr;
  const int64_t* ibase = M.win_ibase;
  for (int64_t w = M.task_w[task]; w < M.nwin; ++w) {
    const int64_t wb = ibase[w], we = ibase[w + 1];
    if (wb >= ie) break;
    const int64_t pb = max(ib, wb), pe = min(ie, we);
    if (pe <= pb) continue;
    const int64_t L = w * M.S;
    const int64_t Sw = min(M.S, M.nkeys - L);
    uint4* z = reinterpret_cast<uint4*>(smem_raw);
    const int nz = (int)((Sw + DENSE_DUMMY) * (int64_t)sizeof(T) / 16);
    __syncthreads();   // the previous piece's flush has read the window
    for (int i = tid; i < nz; i += BS) z[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    const uint32_t S8 = (uint32_t)(Sw * 8);
    // 128-bit: the high words follow the low words (and their discard slots)
    const int64_t hw = Sw + DENSE_DUMMY;
    const uint32_t hi8 = (uint32_t)(hw * 8);
    if constexpr (std::is_same<T, double>::value) {
      if (trunc) run_items<T, 3, BS, true>(M, pb, pe, L, S8, base, hi8);
      else run_items<T, 3, BS, false>(M, pb, pe, L, S8, base, hi8);
    } else if constexpr (std::is_same<T, I128>::value) {
      if (trunc) run_items<T, 5, BS, true>(M, pb, pe, L, S8, base, hi8);
      else run_items<T, 5, BS, false>(M, pb, pe, L, S8, base, hi8);
    } else if (trunc) {   // truncated products: the narrowest kind, or general int64
      if (narrow & 4u) run_items<T, 4, BS, true>(M, pb, pe, L, S8, base, hi8);
      else run_items<T, 0, BS, true>(M, pb, pe, L, S8, base, hi8);
    } else {
      if (narrow & 4u) run_items<T, 4, BS, false>(M, pb, pe, L, S8, base, hi8);
      else if (narrow & 2u) run_items<T, 2, BS, false>(M, pb, pe, L, S8, base, hi8);
      else if (narrow & 1u) run_items<T, 1, BS, false>(M, pb, pe, L, S8, base, hi8);
      else run_items<T, 0, BS, false>(M, pb, pe, L, S8, base, hi8);
    }
    __syncthreads();
    flush_window<T, BS>(M, smem_raw, L, Sw, hw, !M.accumulate && pb == wb && pe == we);
  }
}

// ------------------------------------------------------------------ split windows
struct CombineArgs {
  const int64_t* win_split;
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
  if (!C.win_split[w]) return;
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
  Mailbox* mb;      // optional: the count is posted here as soon as it is known
  uint64_t seq;
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
    // errors of this call, and any latched on the context by an earlier
    // asynchronous call (an encode that found an exponent out of range)
    uint32_t e = A.meta->err | A.meta->seg_err[0] | A.meta->seg_err[1] | *A.ctx_err;
    if (total > A.out_cap) e |= ERR_CAPACITY;
    const int64_t n = e ? -(int64_t)first_error(e) : total;
    if (e) atomicOr(A.ctx_err, e);
    *A.out_n = n;
    // the waiting host needs only the count; the copy follows in stream order
    if (A.mb) post_count(A.mb, A.seq, n, e);
  }
}

struct CopyArgs {
  int64_t out_cap;
  const int64_t* ccount;
  const int64_t* coff;    // from the scan kernel (not used when the copy scans)
  const int64_t* stage_k;
  const int64_t* stage_c;
  int64_t* out_k;
  int64_t* out_c;
  int32_t* out_x;   // optional: decoded exponents instead of codes
  DevLayout L;
  const int64_t* out_n;   // the scan's count: nothing is written after an error
  // a copy that scans itself: the inputs and outputs of the scan kernel
  const Meta* meta;
  int64_t nchunk;
  int64_t* out_n_w;
  uint32_t* ctx_err;
  Mailbox* mb;
  uint64_t seq;
};

// Chunks up to which the copy kernel also does the scan's work (each of its
// workgroups sums the counts of the chunks before its own), saving a launch.
constexpr int64_t COPY_SCAN_MAX = 4096;

template <bool DECODE, typename T, bool SCAN>
__global__ void __launch_bounds__(256) k_dense_copy(CopyArgs C) {
  const int64_t c = blockIdx.x;
  int64_t off;
  if constexpr (SCAN) {
    // this chunk's offset and the total, from the chunk counts
    __shared__ int64_t s_wave[2][4];
    int64_t before = 0, all = 0;
    for (int64_t k = threadIdx.x; k < C.nchunk; k += 256) {
      const int64_t v = C.ccount[k];
      all += v;
      if (k < c) before += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      before += __shfl_xor(before, o);
      all += __shfl_xor(all, o);
    }
    if ((threadIdx.x & 63) == 0) {
      s_wave[0][threadIdx.x >> 6] = before;
      s_wave[1][threadIdx.x >> 6] = all;
    }
    __syncthreads();
    off = s_wave[0][0] + s_wave[0][1] + s_wave[0][2] + s_wave[0][3];
    const int64_t total = s_wave[1][0] + s_wave[1][1] + s_wave[1][2] + s_wave[1][3];
    // The product's own checks, taken by every workgroup on the same inputs
    // (written by earlier kernels of this stream), decide whether anything
    // is copied.  The context's latched status may change while the copy
    // runs (another stream on the same context), so only workgroup 0 reads
    // it, for the count it posts: a product is then either reported failed
    // or complete, never short.
    uint32_t own = C.meta->err | C.meta->seg_err[0] | C.meta->seg_err[1];
    if (total > C.out_cap) own |= ERR_CAPACITY;
    if (c == 0 && threadIdx.x == 0) {
      const uint32_t e = own | *C.ctx_err;
      const int64_t n = e ? -(int64_t)first_error(e) : total;
      if (own) atomicOr(C.ctx_err, own);
      *C.out_n_w = n;
      if (C.mb) post_count(C.mb, C.seq, n, e);   // the waiting host needs only the count
    }
    if (own) return;
  } else {
    if (*C.out_n < 0) return;
    off = C.coff[c];
  }
  const int64_t n = C.ccount[c];
  const int64_t* sk = C.stage_k + c * DENSE_CHUNK;
  const T* sc = reinterpret_cast<const T*>(C.stage_c) + c * DENSE_CHUNK;
  T* out_c = reinterpret_cast<T*>(C.out_c);
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    const int64_t q = off + r;
    if (q < C.out_cap) {
      if constexpr (DECODE) {
        int32_t ex[KP_MAX_VARS];
        decode_x(C.L, (uint64_t)sk[r], ex);
        for (int v = 0; v < C.L.nx; ++v) C.out_x[q * C.L.nx + v] = ex[v];
      } else {
        C.out_k[q] = sk[r];
      }
      out_c[q] = sc[r];
    }
  }
}

// Raises the window kernel's dynamic LDS limit and checks that it has no
// static LDS (its window must start at LDS address 0).
template <typename T, int BS>
hipError_t set_lds_limit() {
  const void* f = reinterpret_cast<const void*>(&k_dense_mul<T, BS>);
  hipFuncAttributes at{};
  hipError_t e = hipFuncGetAttributes(&at, f);
  if (e != hipSuccess) return e;
  if (at.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)DENSE_LDS_BYTES);
}

}  // namespace

int dense_bucket_shift(int64_t maxcode, int64_t n) {
  // about two buckets per term (at least 4096, at most DENSE_MAX_BUCKETS):
  // fine enough for the row ranges, small enough for a quick scan
  const int64_t want = std::min(DENSE_MAX_BUCKETS, std::max((int64_t)4096, 2 * n));
  int s = 0;
  while (((maxcode >> s) + 1) > want) ++s;
  return s;
}

// Kernel attributes (dynamic LDS limits), set once per process before any
// launch, so that no launch (or graph capture) has to set them.
hipError_t dense_setup() {
  static bool attrs = false;
  if (!attrs) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_prep),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(DENSE_MAX_BUCKETS * 4));
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_items),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)ITEMS_LDS_BYTES);
    if (e == hipSuccess) e = set_lds_limit<int64_t, 256>();
    if (e == hipSuccess) e = set_lds_limit<int64_t, 512>();
    if (e == hipSuccess) e = set_lds_limit<int64_t, 1024>();
    if (e == hipSuccess) e = set_lds_limit<double, 256>();
    if (e == hipSuccess) e = set_lds_limit<double, 512>();
    if (e == hipSuccess) e = set_lds_limit<double, 1024>();
    if (e == hipSuccess) e = set_lds_limit<I128, 256>();
    if (e == hipSuccess) e = set_lds_limit<I128, 512>();
    if (e == hipSuccess) e = set_lds_limit<I128, 1024>();
    if (e != hipSuccess) return e;
    attrs = true;
  }
  return hipSuccess;
}

hipError_t launch_dense_laurent(const DensePlan& P, const DenseBufs& B, kp_dtype dt, hipStream_t s) {
  hipError_t e0 = dense_setup();
  if (e0 != hipSuccess) return e0;
  PrepArgs pa{};
  pa.seg[0] = PrepSeg{B.a_keys_in, B.a_coef_in, B.na, P.shiftA, P.nbkA, P.maxcodeA, B.apk, B.ac,
                      B.rank_a, B.bstart, nullptr, nullptr, nullptr, 0, B.a_sa_in, B.a_sa};
  pa.seg[1] = PrepSeg{B.b_keys_in, B.b_coef_in, B.nb, P.shiftB, P.nbkB, P.maxcodeB, B.bpk, B.bc,
                      B.rank_b, B.bstartB, B.tmin, B.tmax, B.ccount, P.nchunk, B.b_tb_in, B.b_tb};
  pa.meta = B.meta;
  pa.is_i64 = dt != KP_F64;
  const size_t hist_bytes = (size_t)std::max(P.nbkA, P.nbkB) * 4;
  hipLaunchKernelGGL(k_dense_prep, dim3(2), dim3(PREP_BLOCK), hist_bytes, s, pa);
  const int64_t blocksA = (B.na + SCATTER_BLOCK - 1) / SCATTER_BLOCK;
  const int64_t blocksB = (B.nb + SCATTER_BLOCK - 1) / SCATTER_BLOCK;
  hipLaunchKernelGGL(k_dense_scatter, dim3((unsigned)(blocksA + blocksB)), dim3(SCATTER_BLOCK), 0,
                     s, pa, blocksA);

  PlanArgs pl{P.S, P.nwin, P.ntiles, P.nkeys, B.nb, P.target_tasks, P.min_work, P.items_cap,
              ITEMS_LDS_BYTES, P.accumulate,
              B.bstart, P.shiftA, P.nbkA, B.tmin, B.tmax, B.win, B.recs, B.items, B.task_w,
              B.task_begin, B.dense, B.meta, coef_words(dt)};
  hipLaunchKernelGGL(k_dense_count, dim3((unsigned)P.nwin), dim3(PLAN_BLOCK), 0, s, pl);
  hipLaunchKernelGGL(k_dense_items, dim3((unsigned)P.nwin), dim3(PLAN_BLOCK),
                     (size_t)ITEMS_LDS_BYTES, s, pl);

  const int64_t W1 = P.nwin + 1;
  MulArgs ma{B.meta, B.apk, B.ac, B.bpk, B.bc, B.nb, P.S, P.nwin, P.nkeys, B.items, B.task_w,
             B.task_begin, B.win + W_IBASE * W1, P.accumulate, B.dense, B.stage_k, B.stage_c,
             B.ccount, B.a_sa_in ? B.a_sa : nullptr, B.b_tb_in ? B.b_tb : nullptr};
  const size_t lds = (size_t)(P.S + DENSE_DUMMY) * 8 * coef_words(dt);
  const unsigned grid = (unsigned)P.max_tasks;
  if (B.ev0) (void)hipEventRecord(B.ev0, s);
#define KP_DENSE_LAUNCH(TT, BSZ) \
  hipLaunchKernelGGL((k_dense_mul<TT, BSZ>), dim3(grid), dim3(BSZ), lds, s, ma)
  if (dt == KP_F64) {
    if (P.block == 256) KP_DENSE_LAUNCH(double, 256);
    else if (P.block == 512) KP_DENSE_LAUNCH(double, 512);
    else KP_DENSE_LAUNCH(double, 1024);
  } else if (dt == KP_I128) {
    if (P.block == 256) KP_DENSE_LAUNCH(I128, 256);
    else if (P.block == 512) KP_DENSE_LAUNCH(I128, 512);
    else KP_DENSE_LAUNCH(I128, 1024);
  } else {
    if (P.block == 256) KP_DENSE_LAUNCH(int64_t, 256);
    else if (P.block == 512) KP_DENSE_LAUNCH(int64_t, 512);
    else KP_DENSE_LAUNCH(int64_t, 1024);
  }
#undef KP_DENSE_LAUNCH
  if (B.ev1) (void)hipEventRecord(B.ev1, s);
  if (P.accumulate) return hipGetLastError();   // the caller reads the accumulator

  CombineArgs cb{B.win + W_SPLIT * W1, P.nwin, P.S, P.nkeys, B.dense, B.stage_k, B.stage_c,
                 B.ccount};
  const unsigned cgrid = (unsigned)(P.nwin * (P.S / DENSE_CHUNK));
  if (dt == KP_F64)
    hipLaunchKernelGGL(k_dense_combine<double>, dim3(cgrid), dim3(COMBINE_BLOCK), 0, s, cb);
  else if (dt == KP_I128)
    hipLaunchKernelGGL(k_dense_combine<I128>, dim3(cgrid), dim3(COMBINE_BLOCK), 0, s, cb);
  else
    hipLaunchKernelGGL(k_dense_combine<int64_t>, dim3(cgrid), dim3(COMBINE_BLOCK), 0, s, cb);

  CopyArgs ca{B.out_cap, B.ccount, B.coff, B.stage_k, B.stage_c, B.out_k,
              reinterpret_cast<int64_t*>(B.out_c), B.out_exps, B.dec, B.out_n,
              B.meta, P.nchunk, B.out_n, B.ctx_err, B.mb, B.seq};
  const bool scan_in_copy = P.nchunk <= COPY_SCAN_MAX;
  if (!scan_in_copy) {
    ScanArgs sa{B.meta, P.nchunk, B.out_cap, B.ccount, B.coff, B.out_n, B.ctx_err, B.mb, B.seq};
    hipLaunchKernelGGL(k_dense_scan, dim3(1), dim3(1024), 0, s, sa);
  }
  const dim3 cg((unsigned)P.nchunk);
#define KP_COPY(DEC, TT)                                                                        \
  do {                                                                                          \
    if (scan_in_copy) hipLaunchKernelGGL((k_dense_copy<DEC, TT, true>), cg, dim3(256), 0, s, ca); \
    else hipLaunchKernelGGL((k_dense_copy<DEC, TT, false>), cg, dim3(256), 0, s, ca);           \
  } while (0)
  if (dt == KP_I128) {
    if (B.out_exps) KP_COPY(true, I128);
    else KP_COPY(false, I128);
  } else {
    if (B.out_exps) KP_COPY(true, int64_t);
    else KP_COPY(false, int64_t);
  }
#undef KP_COPY
  return hipGetLastError();
}

}  // namespace kp
