// kp_codec.hip -- per-variable min/max, Kronecker encode and decode kernels,
// plus the small bookkeeping kernels shared by the multiply paths.
//
// Encode and decode apply the generalised Kronecker map of Section 2
// (c(e) = c.e - chi with per-variable widths and negative offsets); the
// per-term arithmetic is in kp_internal.h so the host twins run the same map.
#include <algorithm>
#include <climits>

#include "kp_internal.h"

namespace kp {

namespace {

constexpr int CODEC_BLOCK = 256;

__global__ void __launch_bounds__(CODEC_BLOCK)
k_minmax_init(int32_t nv, int32_t* out, int empty) {
  int v = threadIdx.x;
  if (v < nv) {
    out[v] = empty ? 0 : INT_MAX;
    out[nv + v] = empty ? -1 : INT_MIN;
  }
}

// Each thread folds a strided set of rows into per-variable registers, then
// the block reduces through LDS and folds into `out` with atomics.
__global__ void __launch_bounds__(CODEC_BLOCK)
k_minmax(int64_t n, int32_t nv, const int32_t* __restrict__ vals, int32_t* out) {
  __shared__ int32_t smin[KP_MAX_VARS][CODEC_BLOCK / 64];
  __shared__ int32_t smax[KP_MAX_VARS][CODEC_BLOCK / 64];
  int32_t lo[KP_MAX_VARS], hi[KP_MAX_VARS];
#pragma unroll
  for (int v = 0; v < KP_MAX_VARS; ++v) {
    lo[v] = INT_MAX;
    hi[v] = INT_MIN;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int v = 0; v < KP_MAX_VARS; ++v) {
      if (v < nv) {
        int32_t x = vals[i * nv + v];
        lo[v] = min(lo[v], x);
        hi[v] = max(hi[v], x);
      }
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
  if (threadIdx.x < nv) {
    int v = threadIdx.x;
    int32_t a = INT_MAX, b = INT_MIN;
    for (int w = 0; w < CODEC_BLOCK / 64; ++w) {
      a = min(a, smin[v][w]);
      b = max(b, smax[v][w]);
    }
    atomicMin(&out[v], a);
    atomicMax(&out[nv + v], b);
  }
}

// Boxes of several exponent arrays in one launch.  Every workgroup posts its
// partial box (per variable min and max over its share of the words) to the
// host mailbox, each word tagged with the low 32 bits of the call's sequence
// number; the host waits for all the tagged words and combines them.  No
// device atomics, no last-workgroup step, no fence: each post is one 64-bit
// store.  One workgroup per array handles arrays of up to BOX_ONE_ROWS rows;
// longer arrays take up to BOX_PARTS workgroups each (blockIdx.y = array).
__device__ __forceinline__ void post_box(const BoxArgs& A, int g, int part, int r, int32_t v) {
  const uint64_t w = ((uint64_t)(uint32_t)A.seq << 32) | (uint32_t)v;
  __hip_atomic_store(&A.mb->box_part[g][part][r], w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

constexpr int BOX_BLOCK = 1024;
constexpr int64_t BOX_ONE_ROWS = 2048;

__global__ void __launch_bounds__(BOX_BLOCK) k_boxes_one(BoxArgs A) {
  __shared__ int32_t smin[KP_MAX_VARS][BOX_BLOCK / 64];
  __shared__ int32_t smax[KP_MAX_VARS][BOX_BLOCK / 64];
  const int g = blockIdx.x;
  const int64_t n = A.n[g];
  const int32_t nv = A.nv[g];
  const int32_t* __restrict__ vals = A.vals[g];
  int32_t lo[KP_MAX_VARS], hi[KP_MAX_VARS];
#pragma unroll
  for (int v = 0; v < KP_MAX_VARS; ++v) {
    lo[v] = INT_MAX;
    hi[v] = INT_MIN;
  }
  // the block's rows as one flat run of n * nv words, BOX_UNROLL loads in
  // flight per thread; word w belongs to variable w % nv
  constexpr int BOX_UNROLL = 8;
  const int64_t words = n * nv;
  for (int64_t w0 = threadIdx.x; w0 < words; w0 += (int64_t)BOX_BLOCK * BOX_UNROLL) {
    int32_t x[BOX_UNROLL];
#pragma unroll
    for (int u = 0; u < BOX_UNROLL; ++u) {
      const int64_t w = w0 + (int64_t)u * BOX_BLOCK;
      x[u] = w < words ? vals[w] : 0;
    }
    int v = (int)(w0 % nv);
    const int step = BOX_BLOCK % nv;
#pragma unroll
    for (int u = 0; u < BOX_UNROLL; ++u) {
      const int64_t w = w0 + (int64_t)u * BOX_BLOCK;
      if (w < words) {
#pragma unroll
        for (int q = 0; q < KP_MAX_VARS; ++q)
          if (q == v) {
            lo[q] = min(lo[q], x[u]);
            hi[q] = max(hi[q], x[u]);
          }
      }
      v += step;
      if (v >= nv) v -= nv;
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
      for (int w = 0; w < BOX_BLOCK / 64; ++w) r = is_max ? max(r, smax[v][w]) : min(r, smin[v][w]);
      post_box(A, g, 0, threadIdx.x, r);
    }
  }
}

__global__ void __launch_bounds__(CODEC_BLOCK) k_boxes(BoxArgs A) {
  __shared__ int32_t smin[KP_MAX_VARS][CODEC_BLOCK / 64];
  __shared__ int32_t smax[KP_MAX_VARS][CODEC_BLOCK / 64];
  const int g = blockIdx.y;
  const int64_t n = A.n[g];
  const int32_t nv = A.nv[g];
  const int32_t* __restrict__ vals = A.vals[g];
  int32_t lo[KP_MAX_VARS], hi[KP_MAX_VARS];
#pragma unroll
  for (int v = 0; v < KP_MAX_VARS; ++v) {
    lo[v] = INT_MAX;
    hi[v] = INT_MIN;
  }
  // the rows as one flat run of n * nv words (word w belongs to variable
  // w % nv), BOX_UNROLL loads in flight per thread: one round of loads when
  // the grid is sized for it
  constexpr int BOX_UNROLL = 8;
  const int64_t words = n * nv;
  const int64_t T = (int64_t)gridDim.x * CODEC_BLOCK;
  const int step = (int)(T % nv);
  for (int64_t w0 = (int64_t)blockIdx.x * CODEC_BLOCK + threadIdx.x; w0 < words;
       w0 += T * BOX_UNROLL) {
    int32_t x[BOX_UNROLL];
#pragma unroll
    for (int u = 0; u < BOX_UNROLL; ++u) {
      const int64_t w = w0 + (int64_t)u * T;
      x[u] = w < words ? vals[w] : 0;
    }
    int v = (int)(w0 % nv);
#pragma unroll
    for (int u = 0; u < BOX_UNROLL; ++u) {
      if (w0 + (int64_t)u * T < words) {
#pragma unroll
        for (int q = 0; q < KP_MAX_VARS; ++q)
          if (q == v) {
            lo[q] = min(lo[q], x[u]);
            hi[q] = max(hi[q], x[u]);
          }
      }
      v += step;
      if (v >= nv) v -= nv;
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
      for (int w = 0; w < CODEC_BLOCK / 64; ++w) r = is_max ? max(r, smax[v][w]) : min(r, smin[v][w]);
      post_box(A, g, blockIdx.x, threadIdx.x, r);
    }
  }
}

__global__ void k_post_count(const int64_t* out_n, const uint32_t* ctx_err, Mailbox* mb,
                             uint64_t seq) {
  if (threadIdx.x != 0) return;
  post_count(mb, seq, *out_n, *ctx_err);
}

__device__ __forceinline__ uint32_t encode_row(const DevLayout& L, int64_t r,
                                               const int32_t* __restrict__ x,
                                               const int32_t* __restrict__ y,
                                               const uint8_t* __restrict__ t,
                                               int64_t* __restrict__ kx, int64_t* __restrict__ ky) {
  int32_t ex[KP_MAX_VARS], jy[KP_MAX_VARS];
  for (int v = 0; v < L.nx; ++v) ex[v] = x[r * L.nx + v];
  for (int v = 0; v < L.ny; ++v) jy[v] = y[r * L.ny + v];
  int64_t a = 0, b = 0;
  const uint32_t e = encode_term(L, ex, jy, L.ny > 0 ? t[r] : 0, &a, &b);
  kx[r] = a;
  if (L.ny > 0) ky[r] = b;
  return e;
}

// Weighted degree sum_v w_v e_v of a factor term from its code (digits over
// the product widths, offset by the factor's box minimum).
__device__ __forceinline__ int64_t code_degree(const DevLayout& L, uint64_t q, const int32_t* w) {
  int64_t deg = 0;
  for (int v = 0; v < L.nx; ++v) {
    const uint64_t qq = fdiv(q, L.dx[v]);
    deg += (int64_t)w[v] * ((int64_t)(q - qq * L.dx[v].d) + L.fmin[v]);
    q = qq;
  }
  return deg;
}

// Truncation tables: for a term of A its slack D - deg, for a term of B its
// degree, both as int32 (a pair is kept iff deg_b <= slack_a).  Exact while
// every |deg| <= 2^30, else ERR_RANGE; slacks outside int32 are clamped
// (they then decide the same way for every |deg_b| <= 2^30).
__global__ void __launch_bounds__(CODEC_BLOCK)
k_degrees(DevLayout LA, DevLayout LB, TruncSpec T, int64_t na, int64_t nb,
          const int64_t* __restrict__ ak, const int64_t* __restrict__ bk,
          int32_t* __restrict__ sa, int32_t* __restrict__ tb, uint32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t e = 0;
  constexpr int64_t LIM = (int64_t)1 << 30;
  if (i < na) {
    const int64_t d = code_degree(LA, (uint64_t)ak[i], T.w);
    if (d > LIM || d < -LIM) e = ERR_RANGE;
    sa[i] = (int32_t)max((int64_t)INT_MIN, min((int64_t)INT_MAX, T.max_degree - d));
  } else if (i < na + nb) {
    const int64_t d = code_degree(LB, (uint64_t)bk[i - na], T.w);
    if (d > LIM || d < -LIM) e = ERR_RANGE;
    tb[i - na] = (int32_t)max(-LIM, min(LIM, d));
  }
  const uint32_t any = wave_or(e);
  if (any && (threadIdx.x & 63) == 0) atomicOr(err, any);
}

// Both factors in one launch: rows [0, na) of A, then [na, na + nb) of B.
__global__ void __launch_bounds__(CODEC_BLOCK)
k_encode2(DevLayout LA, DevLayout LB, int64_t na, int64_t nb, const int32_t* __restrict__ ax,
          const int32_t* __restrict__ ay, const uint8_t* __restrict__ at,
          int64_t* __restrict__ akx, int64_t* __restrict__ aky, const int32_t* __restrict__ bx,
          const int32_t* __restrict__ by, const uint8_t* __restrict__ bt,
          int64_t* __restrict__ bkx, int64_t* __restrict__ bky, uint32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t e = 0;
  if (i < na)
    e = encode_row(LA, i, ax, ay, at, akx, aky);
  else if (i < na + nb)
    e = encode_row(LB, i - na, bx, by, bt, bkx, bky);
  uint32_t any = wave_or(e);
  if (any && (threadIdx.x & 63) == 0) atomicOr(err, any);
}

__global__ void __launch_bounds__(CODEC_BLOCK)
k_encode(DevLayout L, int64_t n, const int32_t* __restrict__ x, const int32_t* __restrict__ y,
         const uint8_t* __restrict__ t, int64_t* __restrict__ kx, int64_t* __restrict__ ky,
         uint32_t* err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t e = 0;
  if (i < n) {
    int32_t ex[KP_MAX_VARS], jy[KP_MAX_VARS];
    for (int v = 0; v < L.nx; ++v) ex[v] = x[i * L.nx + v];
    for (int v = 0; v < L.ny; ++v) jy[v] = y[i * L.ny + v];
    int64_t a = 0, b = 0;
    e = encode_term(L, ex, jy, L.ny > 0 ? t[i] : 0, &a, &b);
    kx[i] = a;
    if (L.ny > 0) ky[i] = b;
  }
  // one atomic per wave that saw an error
  uint32_t any = wave_or(e);
  if (any && (threadIdx.x & 63) == 0) atomicOr(err, any);
}

__device__ __forceinline__ uint32_t decode_one(const DevLayout& L, int poisson, int64_t i,
                                               const int64_t* __restrict__ codes,
                                               int32_t* __restrict__ x, int32_t* __restrict__ y,
                                               uint8_t* __restrict__ t) {
  uint32_t e = 0;
  int64_t c = codes[i];
  int32_t ex[KP_MAX_VARS], jy[KP_MAX_VARS];
  if (c < 0 || c >= L.nkeys) {
    e = ERR_RANGE;
    c = 0;
  }
  uint64_t q = (uint64_t)c;
  if (poisson) {
    t[i] = (uint8_t)(q & 1);
    q >>= 1;
    uint64_t u = fdiv(q, L.dWx);
    uint64_t kx = q - u * (uint64_t)L.Wx;
    decode_x(L, kx, ex);
    decode_y(L, u, jy);
    for (int v = 0; v < L.ny; ++v) y[i * L.ny + v] = jy[v];
  } else {
    decode_x(L, q, ex);
  }
  for (int v = 0; v < L.nx; ++v) x[i * L.nx + v] = ex[v];
  return e;
}

__global__ void __launch_bounds__(CODEC_BLOCK)
k_decode(DevLayout L, int poisson, int64_t n, const int64_t* __restrict__ codes,
         int32_t* __restrict__ x, int32_t* __restrict__ y, uint8_t* __restrict__ t,
         uint32_t* err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t e = 0;
  if (i < n) e = decode_one(L, poisson, i, codes, x, y, t);
  uint32_t any = wave_or(e);
  if (any && (threadIdx.x & 63) == 0) atomicOr(err, any);
}

// Decode of a result whose size is on the device (a multiply's count, or a
// negative status, in which case nothing is decoded); at most `cap` terms.
__global__ void __launch_bounds__(CODEC_BLOCK)
k_decode_n(DevLayout L, int poisson, const int64_t* __restrict__ n_dev, int64_t cap,
           const int64_t* __restrict__ codes, int32_t* __restrict__ x, int32_t* __restrict__ y,
           uint8_t* __restrict__ t, uint32_t* err) {
  const int64_t n = min(*n_dev, cap);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t e = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    e |= decode_one(L, poisson, i, codes, x, y, t);
  uint32_t any = wave_or(e);
  if (any && (threadIdx.x & 63) == 0) atomicOr(err, any);
}

__global__ void k_meta_init(Meta* m) {
  if (threadIdx.x == 0) {
    m->err = 0;
    m->narrow = 3u;
    m->ntasks = 0;
    m->out_count = 0;
    m->amax = 0;
    m->bmax = 0;
    m->nbins = 0;
    m->entries = 0;
    m->pack = 0;
    m->reserve = 0;
  }
}

__global__ void __launch_bounds__(256) k_zero(uint4* p, size_t n16, uint8_t* tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__global__ void k_finalize(const Meta* m, int64_t out_cap, int64_t* out_n, uint32_t* ctx_err) {
  if (threadIdx.x != 0) return;
  // errors of this call, and any latched on the context by an earlier
  // asynchronous call (an encode that found an exponent out of range)
  uint32_t e = m->err | *ctx_err;
  int64_t cnt = m->out_count;
  if (cnt > out_cap) e |= ERR_CAPACITY;
  if (e) {
    atomicOr(ctx_err, e);
    *out_n = -(int64_t)first_error(e);
  } else {
    *out_n = cnt;
  }
}

// Range flags of int64 coefficients: bit0 all fit int32, bit1 all fit in a
// signed 24-bit value (so a product needs only the 24-bit multipliers).
__global__ void __launch_bounds__(256)
k_coef_range(const int64_t* __restrict__ a, int64_t na, const int64_t* __restrict__ b, int64_t nb,
             Meta* m) {
  uint32_t ok = 3u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += stride) {
    int64_t c = i < na ? a[i] : b[i - na];
    if (c < INT_MIN || c > INT_MAX) ok &= ~1u;
    if (c < -(1 << 23) || c >= (1 << 23)) ok &= ~2u;
  }
  uint32_t all = wave_and(ok);
  if ((threadIdx.x & 63) == 0 && all != 3u) atomicAnd(&m->narrow, all);
}

int grid_for(int64_t n, int block, int cap = 1 << 20) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

hipError_t launch_minmax(int64_t n, int32_t nv, const int32_t* vals, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax_init, dim3(1), dim3(64), 0, s, nv, out, n == 0 ? 1 : 0);
  if (n > 0) {
    int g = grid_for(n, CODEC_BLOCK, 2048);
    hipLaunchKernelGGL(k_minmax, dim3(g), dim3(CODEC_BLOCK), 0, s, n, nv, vals, out);
  }
  return hipGetLastError();
}

hipError_t launch_degrees(const DevLayout& LA, const DevLayout& LB, const TruncSpec& T, int64_t na,
                          int64_t nb, const int64_t* ak, const int64_t* bk, int32_t* sa,
                          int32_t* tb, uint32_t* err, hipStream_t s) {
  if (na + nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_degrees, dim3(grid_for(na + nb, CODEC_BLOCK, INT_MAX)), dim3(CODEC_BLOCK), 0,
                     s, LA, LB, T, na, nb, ak, bk, sa, tb, err);
  return hipGetLastError();
}

int box_parts(const BoxArgs& A) {
  int64_t n = 0, words = 0;
  for (int g = 0; g < A.nseg; ++g) {
    n = std::max(n, A.n[g]);
    words = std::max(words, A.n[g] * (int64_t)A.nv[g]);
  }
  if (n <= BOX_ONE_ROWS) return 1;
  return grid_for(words, CODEC_BLOCK * 8, BOX_PARTS);   // one round of 8 words per thread
}

hipError_t launch_boxes(const BoxArgs& A, hipStream_t s) {
  int64_t n = 0;
  for (int g = 0; g < A.nseg; ++g) n = std::max(n, A.n[g]);
  if (n <= BOX_ONE_ROWS)
    hipLaunchKernelGGL(k_boxes_one, dim3(A.nseg), dim3(BOX_BLOCK), 0, s, A);
  else
    hipLaunchKernelGGL(k_boxes, dim3(box_parts(A), A.nseg), dim3(CODEC_BLOCK), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_post_count(const int64_t* out_n, const uint32_t* ctx_err, Mailbox* mb,
                             uint64_t seq, hipStream_t s) {
  hipLaunchKernelGGL(k_post_count, dim3(1), dim3(64), 0, s, out_n, ctx_err, mb, seq);
  return hipGetLastError();
}

hipError_t launch_decode_n(const DevLayout& L, int poisson, const int64_t* n_dev, int64_t cap,
                           const int64_t* codes, int32_t* x, int32_t* y, uint8_t* t, uint32_t* err,
                           hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_decode_n, dim3(grid_for(cap, CODEC_BLOCK, 4096)), dim3(CODEC_BLOCK), 0, s,
                     L, poisson, n_dev, cap, codes, x, y, t, err);
  return hipGetLastError();
}

hipError_t launch_encode(const DevLayout& L, int64_t n, const int32_t* x, const int32_t* y,
                         const uint8_t* t, int64_t* kx, int64_t* ky, uint32_t* err, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_encode, dim3(grid_for(n, CODEC_BLOCK, INT_MAX)), dim3(CODEC_BLOCK), 0, s, L,
                     n, x, y, t, kx, ky, err);
  return hipGetLastError();
}

hipError_t launch_encode2(const DevLayout& LA, const DevLayout& LB, int64_t na, int64_t nb,
                          const int32_t* ax, const int32_t* ay, const uint8_t* at, int64_t* akx,
                          int64_t* aky, const int32_t* bx, const int32_t* by, const uint8_t* bt,
                          int64_t* bkx, int64_t* bky, uint32_t* err, hipStream_t s) {
  if (na + nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_encode2, dim3(grid_for(na + nb, CODEC_BLOCK, INT_MAX)), dim3(CODEC_BLOCK),
                     0, s, LA, LB, na, nb, ax, ay, at, akx, aky, bx, by, bt, bkx, bky, err);
  return hipGetLastError();
}

hipError_t launch_decode(const DevLayout& L, int poisson, int64_t n, const int64_t* codes,
                         int32_t* x, int32_t* y, uint8_t* t, uint32_t* err, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_decode, dim3(grid_for(n, CODEC_BLOCK, INT_MAX)), dim3(CODEC_BLOCK), 0, s, L,
                     poisson, n, codes, x, y, t, err);
  return hipGetLastError();
}

hipError_t launch_meta_init(Meta* m, hipStream_t s) {
  hipLaunchKernelGGL(k_meta_init, dim3(1), dim3(64), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  size_t n16 = bytes / 16, tail = bytes % 16;
  int g = grid_for((int64_t)n16, 256, 8192);
  hipLaunchKernelGGL(k_zero, dim3(g), dim3(256), 0, s, (uint4*)p, n16, (uint8_t*)p + n16 * 16,
                     tail);
  return hipGetLastError();
}

hipError_t launch_finalize(const Meta* m, int64_t out_cap, int64_t* out_n, uint32_t* ctx_err,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, m, out_cap, out_n, ctx_err);
  return hipGetLastError();
}

hipError_t launch_coef_range(const int64_t* a, int64_t na, const int64_t* b, int64_t nb, Meta* m,
                             hipStream_t s) {
  if (na + nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_coef_range, dim3(grid_for(na + nb, 256, 1024)), dim3(256), 0, s, a, na, b,
                     nb, m);
  return hipGetLastError();
}

}  // namespace kp
