// kp_sort.hip -- stable key/value sort of Kronecker-coded factors.
//
// Section 3.1 sorts both factors by exponent (code) so that products walk the
// output in order; here the order is what lets the dense kernel find, by
// binary search, exactly the pairs that land in its window of codes.
//
// Two launches at most:
//  1. each 1024-thread workgroup sorts a chunk of 4096 (key, position) pairs
//     in LDS with a bitonic network (ties broken by position: stable);
//  2. if there is more than one chunk, every element finds its final rank as
//     its rank inside its chunk plus, for every other chunk, the number of
//     keys there that precede it (binary search; earlier chunks count equal
//     keys, later chunks do not), then scatters itself.
// Factors here hold at most a few 1e5 terms, so the O(n * chunks * log)
// second pass costs less than further merge passes would.
#include <climits>

#include "kp_internal.h"

namespace kp {

namespace {

constexpr int SORT_BLOCK = 1024;
constexpr int PER_THREAD = SORT_CHUNK / SORT_BLOCK;

struct SortArgs {
  SortSeg seg[2];
  int64_t chunks0;   // chunks of segment 0; blocks beyond belong to segment 1
};

__device__ inline bool before(int64_t ka, int32_t ia, int64_t kb, int32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

__global__ void __launch_bounds__(SORT_BLOCK) k_sort_chunks(SortArgs args) {
  __shared__ int64_t skey[SORT_CHUNK];
  __shared__ int32_t sidx[SORT_CHUNK];
  const int which = blockIdx.x < args.chunks0 ? 0 : 1;
  const SortSeg& sg = args.seg[which];
  const int64_t chunk = which == 0 ? blockIdx.x : blockIdx.x - args.chunks0;
  const int64_t base = chunk * SORT_CHUNK;
  const int64_t count = min((int64_t)SORT_CHUNK, sg.n - base);
  const int tid = threadIdx.x;

#pragma unroll
  for (int r = 0; r < PER_THREAD; ++r) {
    int p = r * SORT_BLOCK + tid;
    skey[p] = p < count ? sg.keys[base + p] : LLONG_MAX;
    sidx[p] = p;
  }
  __syncthreads();

  // bitonic network over SORT_CHUNK elements, ascending
  for (int k = 2; k <= SORT_CHUNK; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int r = 0; r < PER_THREAD / 2; ++r) {
        int t = r * SORT_BLOCK + tid;                 // pair id in [0, SORT_CHUNK / 2)
        int i = ((t & ~(j - 1)) << 1) | (t & (j - 1)); // lower index of the pair
        int l = i | j;
        bool up = (i & k) == 0;
        int64_t ki = skey[i], kl = skey[l];
        int32_t ii = sidx[i], il = sidx[l];
        bool swap = up ? before(kl, il, ki, ii) : before(ki, ii, kl, il);
        if (swap) {
          skey[i] = kl; skey[l] = ki;
          sidx[i] = il; sidx[l] = ii;
        }
      }
      __syncthreads();
    }
  }

  const bool single = sg.n <= SORT_CHUNK;
#pragma unroll
  for (int r = 0; r < PER_THREAD; ++r) {
    int p = r * SORT_BLOCK + tid;
    if (p >= count) continue;
    int64_t key = skey[p];
    int64_t src = base + sidx[p];
    if (single) {
      int64_t val = sg.vals[src];
      sg.out_keys[p] = key;
      if (sg.out_vals) sg.out_vals[p] = val;
      if (sg.out_pairs) {
        sg.out_pairs[2 * p] = key;
        sg.out_pairs[2 * p + 1] = val;
      }
    } else {
      sg.tmp_keys[base + p] = key;
      sg.tmp_idx[base + p] = (int32_t)src;
    }
  }
}

// number of keys in a[0, n) that are < key (strict) or <= key
__device__ inline int64_t rank_in(const int64_t* __restrict__ a, int64_t n, int64_t key,
                                  bool inclusive) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    int64_t v = a[mid];
    bool go_right = inclusive ? (v <= key) : (v < key);
    if (go_right) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_sort_merge(SortArgs args, int64_t n_total) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_total) return;
  const int which = g < args.seg[0].n ? 0 : 1;
  const SortSeg& sg = args.seg[which];
  if (sg.n <= SORT_CHUNK) return;          // sorted by the first pass already
  if (which == 1) g -= args.seg[0].n;
  const int64_t c = g / SORT_CHUNK;
  const int64_t nch = (sg.n + SORT_CHUNK - 1) / SORT_CHUNK;
  const int64_t key = sg.tmp_keys[g];
  int64_t rank = g - c * SORT_CHUNK;
  for (int64_t o = 0; o < nch; ++o) {
    if (o == c) continue;
    int64_t b = o * SORT_CHUNK;
    int64_t len = min((int64_t)SORT_CHUNK, sg.n - b);
    rank += rank_in(sg.tmp_keys + b, len, key, o < c);
  }
  int64_t val = sg.vals[sg.tmp_idx[g]];
  sg.out_keys[rank] = key;
  if (sg.out_vals) sg.out_vals[rank] = val;
  if (sg.out_pairs) {
    sg.out_pairs[2 * rank] = key;
    sg.out_pairs[2 * rank + 1] = val;
  }
}

}  // namespace

size_t sort_tmp_bytes(int64_t n) {
  if (n <= SORT_CHUNK) return 0;
  return (size_t)n * (sizeof(int64_t) + sizeof(int32_t));
}

hipError_t launch_sort2(const SortSeg& a, const SortSeg& b, hipStream_t s) {
  SortArgs args;
  args.seg[0] = a;
  args.seg[1] = b;
  args.chunks0 = (a.n + SORT_CHUNK - 1) / SORT_CHUNK;
  int64_t chunks1 = (b.n + SORT_CHUNK - 1) / SORT_CHUNK;
  int64_t blocks = args.chunks0 + chunks1;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_chunks, dim3((unsigned)blocks), dim3(SORT_BLOCK), 0, s, args);
  if (a.n > SORT_CHUNK || b.n > SORT_CHUNK) {
    int64_t tot = a.n + b.n;
    hipLaunchKernelGGL(k_sort_merge, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, args,
                       tot);
  }
  return hipGetLastError();
}

}  // namespace kp
