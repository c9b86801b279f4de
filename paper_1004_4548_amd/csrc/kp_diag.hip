// kp_diag.hip -- measurements of the roofline denominators on the device.
//
// The dense window kernel is bound by 64-bit LDS atomic adds.  This probe
// fills every compute unit with one 1024-thread workgroup holding a 128 KiB
// LDS array and times ds_add_u64 at two address patterns: consecutive
// 8-byte slots per wavefront (no bank conflicts) and pseudo-random slots
// (the conflicts of data-dependent addresses).
#include "kp_internal.h"

namespace kp {

namespace {

constexpr int PROBE_BLOCK = 1024;
constexpr int PROBE_SLOTS = 16384;   // 128 KiB of 8-byte counters
constexpr int PROBE_UNROLL = 16;

template <int RANDOM>
__global__ void __launch_bounds__(PROBE_BLOCK) k_lds_atomic_probe(unsigned long long* out, int iters) {
  __shared__ unsigned long long buf[PROBE_SLOTS];
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
      atomicAdd(&buf[s], 1ull);
    }
  }
  __syncthreads();
  if (tid == 0) out[blockIdx.x % 16] = buf[0] + buf[PROBE_SLOTS - 1];   // keeps the adds
}

}  // namespace

hipError_t probe_lds_atomic(int random, int blocks, int iters, unsigned long long* sink,
                            float* ms, hipStream_t s) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) {
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the first run warms up
      e = hipEventRecord(a, s);
      if (random)
        hipLaunchKernelGGL(k_lds_atomic_probe<1>, dim3(blocks), dim3(PROBE_BLOCK), 0, s, sink,
                           iters);
      else
        hipLaunchKernelGGL(k_lds_atomic_probe<0>, dim3(blocks), dim3(PROBE_BLOCK), 0, s, sink,
                           iters);
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
