// kp_diag.hip -- measurements of the roofline denominators on the device.
//
// The dense window kernel is bound by LDS atomic adds.  This probe fills
// every compute unit with one 1024-thread workgroup holding a 128 KiB LDS
// array and times atomic adds of 64-bit or 32-bit counters at two address
// patterns: consecutive counters per wavefront (no bank conflicts) and
// pseudo-random counters (the conflicts of data-dependent addresses).  A
// fifth pattern times the 128-bit accumulation of exact products: at random
// slots of two 64 KiB word arrays, a returning add on the low word, then an
// add of the carry into the high word, eight pairs in flight per lane.
#include "kp_internal.h"

namespace kp {

namespace {

constexpr int PROBE_BLOCK = 1024;
constexpr int PROBE_BYTES = 131072;
constexpr int PROBE_UNROLL = 16;

template <typename T, int RANDOM>
__global__ void __launch_bounds__(PROBE_BLOCK) k_lds_atomic_probe(unsigned long long* out, int iters) {
  constexpr int PROBE_SLOTS = PROBE_BYTES / (int)sizeof(T);
  __shared__ T buf[PROBE_SLOTS];
  const int tid = threadIdx.x;
  for (int i = tid; i < PROBE_SLOTS; i += PROBE_BLOCK) buf[i] = 0;
  __syncthreads();
  uint32_t slot[PROBE_UNROLL];
#pragma unroll
  for (int u = 0; u < PROBE_UNROLL; ++u) {
    if (RANDOM) {
      uint32_t h = (uint32_t)(tid * PROBE_UNROLL + u) * 2654435761u + blockIdx.x * 40503u;
      h ^= h >> 15;
      h *= 2246822519u;
      h ^= h >> 13;
      slot[u] = h & (PROBE_SLOTS - 1);
    } else {
      slot[u] = (uint32_t)(u * PROBE_BLOCK + tid) & (PROBE_SLOTS - 1);
    }
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; ++u) {
      const uint32_t s = RANDOM ? ((slot[u] + (uint32_t)it * 977u) & (PROBE_SLOTS - 1)) : slot[u];
      atomicAdd(&buf[s], (T)1);
    }
  }
  __syncthreads();
  if (tid == 0) out[blockIdx.x % 16] = (unsigned long long)buf[0] + buf[PROBE_SLOTS - 1];   // keeps the adds
}

constexpr int PAIR_WORDS = PROBE_BYTES / 16;   // slots of each word array
constexpr int PAIR_UNROLL = 8;

__global__ void __launch_bounds__(PROBE_BLOCK) k_lds_pair_probe(unsigned long long* out, int iters) {
  __shared__ unsigned long long lo[PAIR_WORDS];
  __shared__ unsigned long long hi[PAIR_WORDS];
  const int tid = threadIdx.x;
  for (int i = tid; i < PAIR_WORDS; i += PROBE_BLOCK) lo[i] = hi[i] = 0;
  __syncthreads();
  uint32_t slot[PAIR_UNROLL];
#pragma unroll
  for (int u = 0; u < PAIR_UNROLL; ++u) {
    uint32_t h = (uint32_t)(tid * PAIR_UNROLL + u) * 2654435761u + blockIdx.x * 40503u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    slot[u] = h & (PAIR_WORDS - 1);
  }
  const unsigned long long v = 0xF0000000F0000000ull + (unsigned long long)tid;
  for (int it = 0; it < 2 * iters; ++it) {
    unsigned long long old[PAIR_UNROLL];
    uint32_t s[PAIR_UNROLL];
#pragma unroll
    for (int u = 0; u < PAIR_UNROLL; ++u) {
      s[u] = (slot[u] + (uint32_t)it * 977u) & (PAIR_WORDS - 1);
      old[u] = atomicAdd(&lo[s[u]], v);
    }
#pragma unroll
    for (int u = 0; u < PAIR_UNROLL; ++u) atomicAdd(&hi[s[u]], (old[u] + v < old[u]) ? 2ull : 1ull);
  }
  __syncthreads();
  if (tid == 0) out[blockIdx.x % 16] = lo[0] + hi[PAIR_WORDS - 1];   // keeps the adds
}

}  // namespace

// pattern: 0/1 = 64-bit consecutive/random, 2/3 = 32-bit consecutive/random,
// 4 = random 128-bit carry pairs (16 pairs per lane per iteration, as the
// other patterns make 16 adds).
hipError_t probe_lds_atomic(int pattern, int blocks, int iters, unsigned long long* sink,
                            float* ms, hipStream_t s) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) {
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the first run warms up
      e = hipEventRecord(a, s);
      switch (pattern) {
        case 0:
          hipLaunchKernelGGL((k_lds_atomic_probe<unsigned long long, 0>), dim3(blocks),
                             dim3(PROBE_BLOCK), 0, s, sink, iters);
          break;
        case 1:
          hipLaunchKernelGGL((k_lds_atomic_probe<unsigned long long, 1>), dim3(blocks),
                             dim3(PROBE_BLOCK), 0, s, sink, iters);
          break;
        case 2:
          hipLaunchKernelGGL((k_lds_atomic_probe<unsigned int, 0>), dim3(blocks), dim3(PROBE_BLOCK),
                             0, s, sink, iters);
          break;
        case 3:
          hipLaunchKernelGGL((k_lds_atomic_probe<unsigned int, 1>), dim3(blocks), dim3(PROBE_BLOCK),
                             0, s, sink, iters);
          break;
        default:
          hipLaunchKernelGGL(k_lds_pair_probe, dim3(blocks), dim3(PROBE_BLOCK), 0, s, sink, iters);
          break;
      }
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess) e = hipEventRecord(b, s);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return e;
}

}  // namespace kp
