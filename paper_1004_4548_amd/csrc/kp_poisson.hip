// kp_poisson.hip -- dense (code-indexed) accumulation of a Poisson product.
//
// Section 2 (eq. werner, with the factor 1/2): a pair of terms with
// trigonometric arguments alpha, beta contributes +-1/2 ca cb to the term of
// alpha - beta and to the term of alpha + beta; the type of both is
// t = ta xor tb (0 cos, 1 sin) and the sign is -1 exactly for the
// difference of cos * sin and for the sum of sin * sin.  Section 3.1's dense
// array then accumulates by code.
//
// The pair's unfolded code (before canonicalisation) is
//   U = kx + Wx * (ky + Hy),  kx = kxa + kxb,  ky = kya -+ kyb,
// a sum of a code of A, kxa + Wx (kya + Hya), and a code of B,
// kxb + Wx (Hyb -+ kyb) (Hya + Hyb = Hy), so the product is a Laurent-style
// product on which the dense window kernel runs unchanged.  To keep the sign
// and type rules out of the inner loop, the code also carries a segment
//   s = 4 piece + 2 ta + tb   (piece 0 = difference, 1 = sum),
// as s * N with N = Wx (2 Hy + 1): A's code gets 2 ta N, each term of B
// appears twice (once per piece) with (4 piece + tb) N.  The accumulated
// array thus holds, per segment, the plain sums of 1/2 ca cb.  The fold pass
// then applies each segment's sign, adds the mirror image (ky -> -ky, which
// keeps cosines and negates sines) into the canonical key of first nonzero
// multiplier positive, drops sines of the zero multiplier vector and writes
// the nonzero terms.
#include "kp_internal.h"

namespace kp {

namespace {

constexpr int PD_BLOCK = 256;

struct PoissonDenseArgs {
  int64_t Wx, N, Hya, Hyb;
  const int64_t* ax;   // A: x codes, trig codes, sine flags, coefficients
  const int64_t* ay;
  const uint8_t* as;
  const double* ac;
  int64_t na;
  const int64_t* bx;
  const int64_t* by;
  const uint8_t* bs;
  const double* bc;
  int64_t nb;
  int64_t* a_codes;    // out: [na]
  double* a_coef;      // out: [na]
  int64_t* b_codes;    // out: [2 nb] (difference pieces, then sum pieces)
  double* b_coef;      // out: [2 nb]
};

__global__ void __launch_bounds__(PD_BLOCK) k_poisson_dense_prep(PoissonDenseArgs P) {
  const int64_t g = (int64_t)blockIdx.x * PD_BLOCK + threadIdx.x;
  if (g < P.na) {
    P.a_codes[g] = P.ax[g] + P.Wx * (P.ay[g] + P.Hya) + 2 * (int64_t)P.as[g] * P.N;
    P.a_coef[g] = P.ac[g];
  } else if (g < P.na + P.nb) {
    const int64_t j = g - P.na;
    const int64_t tb = P.bs[j];
    const double h = 0.5 * P.bc[j];
    P.b_codes[j] = P.bx[j] + P.Wx * (P.Hyb - P.by[j]) + tb * P.N;              // difference
    P.b_codes[P.nb + j] = P.bx[j] + P.Wx * (P.Hyb + P.by[j]) + (4 + tb) * P.N;  // sum
    P.b_coef[j] = h;
    P.b_coef[P.nb + j] = h;
  }
}

// Sign of segment s = 4 piece + 2 ta + tb.
__device__ __forceinline__ double seg_sign(int s) {
  const int piece = s >> 2, ta = (s >> 1) & 1, tb = s & 1;
  const bool neg = piece == 0 ? (!ta && tb) : (ta && tb);
  return neg ? -1.0 : 1.0;
}

struct FoldArgs {
  int64_t Wx, Hy, N;
  const double* acc;   // [8 N] accumulated segments
  Meta* meta;
  int64_t* out_k;
  double* out_c;
  int64_t out_cap;
};

constexpr int FOLD_PER = 8;

// One thread per canonical position q = kx + Wx ky (ky >= 0) and type t.
__global__ void __launch_bounds__(PD_BLOCK) k_poisson_fold(FoldArgs F) {
  __shared__ int64_t s_wave[PD_BLOCK / 64];
  __shared__ int64_t s_base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t npos = F.Wx * (F.Hy + 1);
  const int64_t nkeys = 2 * npos;
  const int64_t chunk = (int64_t)PD_BLOCK * FOLD_PER;
  for (int64_t base = (int64_t)blockIdx.x * chunk; base < nkeys;
       base += (int64_t)gridDim.x * chunk) {
    double val[FOLD_PER];
    uint64_t ball[FOLD_PER];
    int64_t cnt = 0;
#pragma unroll
    for (int r = 0; r < FOLD_PER; ++r) {
      const int64_t key = base + r * PD_BLOCK + threadIdx.x;   // key = 2 q + t
      double v = 0.0;
      if (key < nkeys) {
        const int64_t q = key >> 1;
        const int t = (int)(key & 1);
        const int64_t ky = q / F.Wx, kx = q - ky * F.Wx;
        if (!(t && ky == 0)) {   // sin of the zero multiplier vector vanishes
          const int64_t up = kx + F.Wx * (F.Hy + ky), um = kx + F.Wx * (F.Hy - ky);
          const double mirror = t ? -1.0 : 1.0;
#pragma unroll
          for (int ta = 0; ta < 2; ++ta) {
            const int tb = ta ^ t;
#pragma unroll
            for (int piece = 0; piece < 2; ++piece) {
              const int s = 4 * piece + 2 * ta + tb;
              const double* a = F.acc + (int64_t)s * F.N;
              double sv = a[up];
              if (ky > 0) sv += mirror * a[um];
              v += seg_sign(s) * sv;
            }
          }
        }
      }
      val[r] = v;
      ball[r] = __ballot(v != 0.0);
      cnt += __popcll(ball[r]);
    }
    if (lane == 0) s_wave[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t tot = 0;
      for (int w = 0; w < PD_BLOCK / 64; ++w) tot += s_wave[w];
      s_base = tot ? (int64_t)atomicAdd((unsigned long long*)&F.meta->out_count,
                                        (unsigned long long)tot)
                   : 0;
    }
    __syncthreads();
    int64_t pos = s_base;
    for (int w = 0; w < wave; ++w) pos += s_wave[w];
    const uint64_t lt = (1ull << lane) - 1;
#pragma unroll
    for (int r = 0; r < FOLD_PER; ++r) {
      if (ball[r] & (1ull << lane)) {
        const int64_t p = pos + __popcll(ball[r] & lt);
        if (p < F.out_cap) {
          F.out_k[p] = base + r * PD_BLOCK + threadIdx.x;
          F.out_c[p] = val[r];
        }
      }
      pos += __popcll(ball[r]);
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_poisson_dense_prep(int64_t Wx, int64_t N, int64_t Hya, int64_t Hyb,
                                     const int64_t* ax, const int64_t* ay, const uint8_t* as,
                                     const double* ac, int64_t na, const int64_t* bx,
                                     const int64_t* by, const uint8_t* bs, const double* bc,
                                     int64_t nb, int64_t* a_codes, double* a_coef,
                                     int64_t* b_codes, double* b_coef, hipStream_t s) {
  const int64_t n = na + nb;
  if (n == 0) return hipSuccess;
  PoissonDenseArgs P{Wx, N, Hya, Hyb, ax, ay, as, ac, na, bx, by, bs, bc, nb,
                     a_codes, a_coef, b_codes, b_coef};
  hipLaunchKernelGGL(k_poisson_dense_prep, dim3((unsigned)((n + PD_BLOCK - 1) / PD_BLOCK)),
                     dim3(PD_BLOCK), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_poisson_fold(int64_t Wx, int64_t Hy, int64_t N, const double* acc, Meta* meta,
                               int64_t* out_k, double* out_c, int64_t out_cap, hipStream_t s) {
  const int64_t nkeys = 2 * Wx * (Hy + 1);
  const int64_t chunk = (int64_t)PD_BLOCK * FOLD_PER;
  int64_t blocks = (nkeys + chunk - 1) / chunk;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  FoldArgs F{Wx, Hy, N, acc, meta, out_k, out_c, out_cap};
  hipLaunchKernelGGL(k_poisson_fold, dim3((unsigned)blocks), dim3(PD_BLOCK), 0, s, F);
  return hipGetLastError();
}

}  // namespace kp
