// kp_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously correct CPU multiply of sparse multivariate Laurent
// polynomials and Poisson series, written straight from the definitions in
// Biscani, "Multiplication of sparse Laurent polynomials and Poisson series on
// modern hardware architectures" (ISSAC 2010):
//   * a Poisson series is a Fourier series whose coefficients are Laurent
//     polynomials (Section 1, eq. ps_def);
//   * the product is the schoolbook sum over every pair of terms (Section 3);
//   * a product of two trigonometric factors splits into cos/sin of the sum
//     and of the difference of the arguments (Section 2, eq. werner, read with
//     the factor 1/2 that the printed formulas omit).
//
// It works on exponent tuples in a std::map and never forms a Kronecker code,
// so it shares nothing with the GPU path.  Only the test suite, the smoke
// check and the CPU-baseline leg of the benchmark may load this library; the
// product path never does.
//
// Arithmetic conventions
//   int64 coefficients: products and sums wrap modulo 2^64 (computed in
//     uint64_t, converted back at the end).
//   exact (dtype 2): int64 coefficients whose products are formed exactly in
//     __int128 and summed modulo 2^128 (in unsigned __int128, where
//     wrap-around is defined).  Coefficients are returned as two int64 words
//     (low word, then high word): the exact sum as a two's complement value
//     while |sum| < 2^127, and as an unsigned value for sums in [0, 2^128).
//   fp64 coefficients: each output term carries a Neumaier-compensated sum and
//     the sum of the absolute values of its contributions (used by the parity
//     tolerance |gpu - oracle| <= tol * abs_sum).
//   Terms whose value is exactly zero are erased from the int64 result; in the
//     fp64 result they are kept (the tolerance check needs their abs_sum) and
//     the caller decides.
//
// Parity pins (what fixes this file independently of itself) live in
// tests/test_oracle_pins.py: n-D convolution (scipy) for Laurent products,
// closed forms of the Fateman and Monagan-Pearce benchmarks (Section 5),
// evaluation homomorphisms mod p = 2^61-1 and over F_{p^2}, and the
// trigonometric identities.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <thread>
#include <utility>
#include <vector>

namespace {

constexpr int MAXV = 16;

// ---------------------------------------------------------------- accumulators
struct AccI64 {
  uint64_t v = 0;
  void add(uint64_t x) { v += x; }
};

struct AccI128 {
  unsigned __int128 v = 0;
  void add(__int128 x) { v += (unsigned __int128)x; }
  void add(unsigned __int128 x) { v += x; }
};

// Neumaier's improvement of Kahan summation; abs is the sum of |contribution|.
struct AccF64 {
  double s = 0.0, c = 0.0, abs = 0.0;
  void add_value(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  void add(double x) {
    add_value(x);
    abs += std::fabs(x);
  }
  void merge(const AccF64& o) {
    add_value(o.s);
    add_value(o.c);
    abs += o.abs;
  }
  double value() const { return s + c; }
};

using LKey = std::array<int32_t, MAXV>;             // Laurent exponents
using PKey = std::array<int32_t, 2 * MAXV + 1>;     // x exps, trig mults, sin flag

struct ResultL {
  int nv = 0;
  int dtype = 0;  // 0 int64, 1 fp64, 2 exact (128-bit)
  std::map<LKey, AccI64> mi;
  std::map<LKey, AccF64> mf;
  std::map<LKey, AccI128> mw;
};

struct ResultP {
  int nx = 0, ny = 0;
  std::map<PKey, AccF64> m;
};

LKey lkey(const int32_t* e, int nv) {
  LKey k{};
  for (int v = 0; v < nv; ++v) k[v] = e[v];
  return k;
}

// ------------------------------------------------------------ Laurent product
// P = sum_{(e,c) in A} sum_{(f,d) in B} (c*d) x^(e+f)   (Section 3: schoolbook)
void laurent_rows(ResultL& r, int64_t r0, int64_t r1, const int32_t* ae, const void* ac,
                  int64_t nb, const int32_t* be, const void* bc) {
  const int nv = r.nv;
  for (int64_t i = r0; i < r1; ++i) {
    for (int64_t j = 0; j < nb; ++j) {
      LKey k{};
      for (int v = 0; v < nv; ++v) k[v] = ae[i * nv + v] + be[j * nv + v];
      if (r.dtype == 0) {
        uint64_t x = (uint64_t)((const int64_t*)ac)[i] * (uint64_t)((const int64_t*)bc)[j];
        r.mi[k].add(x);
      } else if (r.dtype == 2) {
        r.mw[k].add((__int128)((const int64_t*)ac)[i] * (__int128)((const int64_t*)bc)[j]);
      } else {
        double x = ((const double*)ac)[i] * ((const double*)bc)[j];
        r.mf[k].add(x);
      }
    }
  }
}

// ------------------------------------------------------------ Poisson product
// One trigonometric term of a product before canonicalisation.
struct TrigPiece {
  std::array<int32_t, MAXV> j;
  int is_sin;
  double sign;
};

// Product-to-sum split of (cos|sin)(ja.y) * (cos|sin)(jb.y).  Each case is the
// textbook identity with its factor 1/2 (applied by the caller):
//   cos a cos b = 1/2 cos(a-b) + 1/2 cos(a+b)
//   cos a sin b = 1/2 sin(a+b) - 1/2 sin(a-b)
//   sin a cos b = 1/2 sin(a-b) + 1/2 sin(a+b)
//   sin a sin b = 1/2 cos(a-b) - 1/2 cos(a+b)
void werner(const int32_t* ja, int sa, const int32_t* jb, int sb, int ny, TrigPiece out[2]) {
  TrigPiece dif{}, sum{};
  for (int v = 0; v < ny; ++v) {
    dif.j[v] = ja[v] - jb[v];
    sum.j[v] = ja[v] + jb[v];
  }
  if (!sa && !sb) {        // cos * cos
    dif.is_sin = 0; dif.sign = +1.0;
    sum.is_sin = 0; sum.sign = +1.0;
  } else if (!sa && sb) {  // cos * sin
    dif.is_sin = 1; dif.sign = -1.0;
    sum.is_sin = 1; sum.sign = +1.0;
  } else if (sa && !sb) {  // sin * cos
    dif.is_sin = 1; dif.sign = +1.0;
    sum.is_sin = 1; sum.sign = +1.0;
  } else {                 // sin * sin
    dif.is_sin = 0; dif.sign = +1.0;
    sum.is_sin = 0; sum.sign = -1.0;
  }
  out[0] = dif;
  out[1] = sum;
}

// Canonical form: the first nonzero multiplier (scanning from index 0) is
// positive.  cos(-t) = cos(t); sin(-t) = -sin(t).  Returns false when the
// piece vanishes (sin of the zero vector).
bool canonicalise(TrigPiece& p, int ny) {
  int first = -1;
  for (int v = 0; v < ny; ++v)
    if (p.j[v] != 0) { first = v; break; }
  if (first < 0) return !p.is_sin;
  if (p.j[first] < 0) {
    for (int v = 0; v < ny; ++v) p.j[v] = -p.j[v];
    if (p.is_sin) p.sign = -p.sign;
  }
  return true;
}

PKey pkey(const int32_t* x, int nx, const std::array<int32_t, MAXV>& j, int ny, int is_sin) {
  PKey k{};
  for (int v = 0; v < nx; ++v) k[v] = x[v];
  for (int v = 0; v < ny; ++v) k[MAXV + v] = j[v];
  k[2 * MAXV] = is_sin;
  return k;
}

void poisson_pair(std::map<PKey, AccF64>& m, int nx, int ny,
                  const int32_t* xa, const int32_t* ya, int sa, double ca,
                  const int32_t* xb, const int32_t* yb, int sb, double cb) {
  int32_t x[MAXV];
  for (int v = 0; v < nx; ++v) x[v] = xa[v] + xb[v];
  TrigPiece pieces[2];
  werner(ya, sa, yb, sb, ny, pieces);
  const double half = 0.5 * (ca * cb);
  for (auto& p : pieces) {
    if (!canonicalise(p, ny)) continue;
    m[pkey(x, nx, p.j, ny, p.is_sin)].add(p.sign * half);
  }
}

void poisson_rows(ResultP& r, int64_t r0, int64_t r1,
                  const int32_t* ax, const int32_t* ay, const uint8_t* as, const double* ac,
                  int64_t nb, const int32_t* bx, const int32_t* by, const uint8_t* bs,
                  const double* bc) {
  const int nx = r.nx, ny = r.ny;
  for (int64_t i = r0; i < r1; ++i)
    for (int64_t j = 0; j < nb; ++j)
      poisson_pair(r.m, nx, ny, ax + i * nx, ay + i * ny, as[i], ac[i],
                   bx + j * nx, by + j * ny, bs[j], bc[j]);
}

// ----------------------------------------------------- mod p = 2^61 - 1 field
constexpr uint64_t P61 = (1ULL << 61) - 1;

uint64_t modp(unsigned __int128 x) {
  uint64_t lo = (uint64_t)(x & P61);
  uint64_t hi = (uint64_t)(x >> 61);
  uint64_t s = lo + (hi & P61) + (uint64_t)(hi >> 61);
  while (s >= P61) s -= P61;
  return s;
}
uint64_t mulp(uint64_t a, uint64_t b) { return modp((unsigned __int128)a * b); }
uint64_t addp(uint64_t a, uint64_t b) { uint64_t s = a + b; return s >= P61 ? s - P61 : s; }
uint64_t subp(uint64_t a, uint64_t b) { return a >= b ? a - b : a + P61 - b; }
uint64_t powp(uint64_t a, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = mulp(r, a);
    a = mulp(a, a);
    e >>= 1;
  }
  return r;
}
uint64_t invp(uint64_t a) { return powp(a, P61 - 2); }  // Fermat
uint64_t from_i64(int64_t c) {
  // exact residue of the signed integer c
  if (c >= 0) return (uint64_t)c % P61;
  uint64_t m = (uint64_t)(-(c + 1)) + 1;  // |c| without overflow
  return subp(0, m % P61);
}
// integer power with a signed exponent (x must be nonzero)
uint64_t spow(uint64_t x, uint64_t xinv, int64_t e) { return e >= 0 ? powp(x, e) : powp(xinv, -e); }

// Exact residue of a finite double: m * 2^k with integer m (|m| < 2^53).
uint64_t from_f64(double d) {
  if (d == 0.0) return 0;
  int ex = 0;
  double fr = std::frexp(d, &ex);                 // d = fr * 2^ex, 0.5 <= |fr| < 1
  int64_t m = (int64_t)std::ldexp(fr, 53);        // exact
  int k = ex - 53;
  uint64_t r = from_i64(m);
  uint64_t two = 2, half = invp(2);
  return k >= 0 ? mulp(r, powp(two, k)) : mulp(r, powp(half, -k));
}

// F_{p^2} = F_p[i]/(i^2 + 1); valid because p = 3 mod 4.
struct G { uint64_t re, im; };
G gmul(G a, G b) {
  return {subp(mulp(a.re, b.re), mulp(a.im, b.im)), addp(mulp(a.re, b.im), mulp(a.im, b.re))};
}
G gadd(G a, G b) { return {addp(a.re, b.re), addp(a.im, b.im)}; }
G gsub(G a, G b) { return {subp(a.re, b.re), subp(a.im, b.im)}; }
G gpow(G a, uint64_t e) {
  G r{1, 0};
  while (e) {
    if (e & 1) r = gmul(r, a);
    a = gmul(a, a);
    e >>= 1;
  }
  return r;
}
G ginv(G a) {  // 1/(x+iy) = (x-iy)/(x^2+y^2)
  uint64_t n = addp(mulp(a.re, a.re), mulp(a.im, a.im));
  uint64_t ni = invp(n);
  return {mulp(a.re, ni), subp(0, mulp(a.im, ni))};
}

}  // namespace

extern "C" {

// ------------------------------------------------------------------ Laurent
// Product of A (na terms) and B (nb terms) restricted to A's rows
// [row_begin, row_end) (row_end < 0 means na).  nthreads > 1 splits those rows
// into contiguous slices, each with a private map, merged in slice order.
void* oracle_laurent_mul(int nv, int dtype, int64_t na, const int32_t* a_exps, const void* a_coef,
                         int64_t nb, const int32_t* b_exps, const void* b_coef,
                         int64_t row_begin, int64_t row_end, int nthreads) {
  if (nv < 0 || nv > MAXV || dtype < 0 || dtype > 2) return nullptr;
  if (row_end < 0 || row_end > na) row_end = na;
  if (row_begin < 0) row_begin = 0;
  if (nthreads < 1) nthreads = 1;
  auto* res = new ResultL;
  res->nv = nv;
  res->dtype = dtype;
  const int64_t rows = std::max<int64_t>(0, row_end - row_begin);
  if (nthreads == 1 || rows < 2) {
    laurent_rows(*res, row_begin, row_end, a_exps, a_coef, nb, b_exps, b_coef);
    return res;
  }
  std::vector<ResultL> part(nthreads);
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) {
    part[t].nv = nv;
    part[t].dtype = dtype;
    int64_t s = row_begin + rows * t / nthreads, e = row_begin + rows * (t + 1) / nthreads;
    th.emplace_back([&, t, s, e] { laurent_rows(part[t], s, e, a_exps, a_coef, nb, b_exps, b_coef); });
  }
  for (auto& x : th) x.join();
  for (int t = 0; t < nthreads; ++t) {
    if (dtype == 0)
      for (auto& kv : part[t].mi) res->mi[kv.first].add(kv.second.v);
    else if (dtype == 2)
      for (auto& kv : part[t].mw) res->mw[kv.first].add(kv.second.v);
    else
      for (auto& kv : part[t].mf) res->mf[kv.first].merge(kv.second);
  }
  return res;
}

// Number of terms: integer results drop exact zeros, fp64 keeps every key touched.
int64_t oracle_laurent_len(void* h) {
  auto* r = (ResultL*)h;
  if (r->dtype == 1) return (int64_t)r->mf.size();
  int64_t n = 0;
  if (r->dtype == 2)
    for (auto& kv : r->mw) n += kv.second.v != 0;
  else
    for (auto& kv : r->mi) n += kv.second.v != 0;
  return n;
}

// Two int64 words (low, high) of a 128-bit value.
void put_i128(unsigned __int128 u, int64_t* out) {
  out[0] = (int64_t)(uint64_t)u;
  out[1] = (int64_t)(uint64_t)(u >> 64);
}

// Key-sorted (lexicographic on exponent 0, 1, ...) result.  abs_sum may be
// null; for int64 it is ignored.
void oracle_laurent_get(void* h, int32_t* exps, void* coef, double* abs_sum) {
  auto* r = (ResultL*)h;
  const int nv = r->nv;
  int64_t t = 0;
  if (r->dtype == 0) {
    for (auto& kv : r->mi) {
      if (kv.second.v == 0) continue;
      for (int v = 0; v < nv; ++v) exps[t * nv + v] = kv.first[v];
      ((int64_t*)coef)[t] = (int64_t)kv.second.v;
      ++t;
    }
  } else if (r->dtype == 2) {
    for (auto& kv : r->mw) {
      if (kv.second.v == 0) continue;
      for (int v = 0; v < nv; ++v) exps[t * nv + v] = kv.first[v];
      put_i128(kv.second.v, (int64_t*)coef + 2 * t);
      ++t;
    }
  } else {
    for (auto& kv : r->mf) {
      for (int v = 0; v < nv; ++v) exps[t * nv + v] = kv.first[v];
      ((double*)coef)[t] = kv.second.value();
      if (abs_sum) abs_sum[t] = kv.second.abs;
      ++t;
    }
  }
}

void oracle_laurent_free(void* h) { delete (ResultL*)h; }

// Coefficient of each queried monomial E, computed one query at a time as
// sum_i ca_i * cb(E - ea_i) with B held in a map from exponents to its terms.
void oracle_laurent_coeff_at(int nv, int dtype, int64_t na, const int32_t* a_exps, const void* a_coef,
                             int64_t nb, const int32_t* b_exps, const void* b_coef, int64_t nq,
                             const int32_t* q_exps, void* out_coef, double* out_abs,
                             int64_t* out_count) {
  std::map<LKey, std::vector<int64_t>> bidx;
  for (int64_t j = 0; j < nb; ++j) bidx[lkey(b_exps + j * nv, nv)].push_back(j);
  for (int64_t q = 0; q < nq; ++q) {
    AccI64 ai;
    AccI128 aw;
    AccF64 af;
    int64_t cnt = 0;
    for (int64_t i = 0; i < na; ++i) {
      LKey k{};
      for (int v = 0; v < nv; ++v) k[v] = q_exps[q * nv + v] - a_exps[i * nv + v];
      auto it = bidx.find(k);
      if (it == bidx.end()) continue;
      for (int64_t j : it->second) {
        ++cnt;
        if (dtype == 0)
          ai.add((uint64_t)((const int64_t*)a_coef)[i] * (uint64_t)((const int64_t*)b_coef)[j]);
        else if (dtype == 2)
          aw.add((__int128)((const int64_t*)a_coef)[i] * (__int128)((const int64_t*)b_coef)[j]);
        else
          af.add(((const double*)a_coef)[i] * ((const double*)b_coef)[j]);
      }
    }
    if (dtype == 0)
      ((int64_t*)out_coef)[q] = (int64_t)ai.v;
    else if (dtype == 2)
      put_i128(aw.v, (int64_t*)out_coef + 2 * q);
    else {
      ((double*)out_coef)[q] = af.value();
      if (out_abs) out_abs[q] = af.abs;
    }
    if (out_count) out_count[q] = cnt;
  }
}

// ------------------------------------------------------------------ Poisson
void* oracle_poisson_mul(int nx, int ny, int64_t na, const int32_t* ax, const int32_t* ay,
                         const uint8_t* as, const double* ac, int64_t nb, const int32_t* bx,
                         const int32_t* by, const uint8_t* bs, const double* bc,
                         int64_t row_begin, int64_t row_end, int nthreads) {
  if (nx < 0 || nx > MAXV || ny < 0 || ny > MAXV) return nullptr;
  if (row_end < 0 || row_end > na) row_end = na;
  if (row_begin < 0) row_begin = 0;
  if (nthreads < 1) nthreads = 1;
  auto* res = new ResultP;
  res->nx = nx;
  res->ny = ny;
  const int64_t rows = std::max<int64_t>(0, row_end - row_begin);
  if (nthreads == 1 || rows < 2) {
    poisson_rows(*res, row_begin, row_end, ax, ay, as, ac, nb, bx, by, bs, bc);
    return res;
  }
  std::vector<ResultP> part(nthreads);
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) {
    part[t].nx = nx;
    part[t].ny = ny;
    int64_t s = row_begin + rows * t / nthreads, e = row_begin + rows * (t + 1) / nthreads;
    th.emplace_back([&, t, s, e] { poisson_rows(part[t], s, e, ax, ay, as, ac, nb, bx, by, bs, bc); });
  }
  for (auto& x : th) x.join();
  for (int t = 0; t < nthreads; ++t)
    for (auto& kv : part[t].m) res->m[kv.first].merge(kv.second);
  return res;
}

int64_t oracle_poisson_len(void* h) { return (int64_t)((ResultP*)h)->m.size(); }

// Key-sorted result: x exponents, then trig multipliers, then the sin flag.
void oracle_poisson_get(void* h, int32_t* x, int32_t* y, uint8_t* is_sin, double* coef,
                        double* abs_sum) {
  auto* r = (ResultP*)h;
  int64_t t = 0;
  for (auto& kv : r->m) {
    for (int v = 0; v < r->nx; ++v) x[t * r->nx + v] = kv.first[v];
    for (int v = 0; v < r->ny; ++v) y[t * r->ny + v] = kv.first[MAXV + v];
    is_sin[t] = (uint8_t)kv.first[2 * MAXV];
    coef[t] = kv.second.value();
    if (abs_sum) abs_sum[t] = kv.second.abs;
    ++t;
  }
}

void oracle_poisson_free(void* h) { delete (ResultP*)h; }

// Coefficient of each queried term (x, j, t), one query at a time.  For every
// term a of A, the only terms of B that can reach the query have x part
// x - xa and a trig vector jb with ja - jb = +-j or ja + jb = +-j; each such
// candidate present in B is multiplied with the full split above and only the
// pieces that land on the query are summed.
void oracle_poisson_coeff_at(int nx, int ny, int64_t na, const int32_t* ax, const int32_t* ay,
                             const uint8_t* as, const double* ac, int64_t nb, const int32_t* bx,
                             const int32_t* by, const uint8_t* bs, const double* bc, int64_t nq,
                             const int32_t* qx, const int32_t* qy, const uint8_t* qs,
                             double* out_coef, double* out_abs, int64_t* out_count) {
  std::map<PKey, std::vector<int64_t>> bidx;
  for (int64_t j = 0; j < nb; ++j) {
    std::array<int32_t, MAXV> jj{};
    for (int v = 0; v < ny; ++v) jj[v] = by[j * ny + v];
    bidx[pkey(bx + j * nx, nx, jj, ny, bs[j])].push_back(j);
  }
  for (int64_t q = 0; q < nq; ++q) {
    std::array<int32_t, MAXV> qj{};
    for (int v = 0; v < ny; ++v) qj[v] = qy[q * ny + v];
    const PKey target = pkey(qx + q * nx, nx, qj, ny, qs[q]);
    AccF64 acc;
    int64_t cnt = 0;
    for (int64_t i = 0; i < na; ++i) {
      int32_t xb[MAXV];
      for (int v = 0; v < nx; ++v) xb[v] = qx[q * nx + v] - ax[i * nx + v];
      // candidates jb: ja - j, j - ja, ja + j, -ja - j  (deduplicated)
      std::vector<std::array<int32_t, MAXV>> cand;
      for (int c = 0; c < 4; ++c) {
        std::array<int32_t, MAXV> jb{};
        for (int v = 0; v < ny; ++v) {
          int32_t ja = ay[i * ny + v], jq = qj[v];
          jb[v] = c == 0 ? ja - jq : c == 1 ? jq - ja : c == 2 ? ja + jq : -ja - jq;
        }
        if (std::find(cand.begin(), cand.end(), jb) == cand.end()) cand.push_back(jb);
      }
      for (auto& jb : cand) {
        for (int tb = 0; tb < 2; ++tb) {
          auto it = bidx.find(pkey(xb, nx, jb, ny, tb));
          if (it == bidx.end()) continue;
          for (int64_t j : it->second) {
            std::map<PKey, AccF64> one;
            poisson_pair(one, nx, ny, ax + i * nx, ay + i * ny, as[i], ac[i], bx + j * nx,
                         by + j * ny, bs[j], bc[j]);
            auto hit = one.find(target);
            if (hit != one.end()) {
              acc.add(hit->second.value());
              ++cnt;
            }
          }
        }
      }
    }
    out_coef[q] = acc.value();
    if (out_abs) out_abs[q] = acc.abs;
    if (out_count) out_count[q] = cnt;
  }
}

// ------------------------------------------------------ evaluation checkers
// sum_t c_t * prod_k r_k^e_tk  mod p (p = 2^61 - 1), int64 coefficients taken
// as exact integers, negative exponents through inverses.  r_k must be nonzero.
uint64_t oracle_laurent_eval_modp_i64(int nv, int64_t n, const int32_t* exps, const int64_t* coef,
                                      const uint64_t* point) {
  uint64_t inv[MAXV];
  for (int v = 0; v < nv; ++v) inv[v] = invp(point[v]);
  uint64_t acc = 0;
  for (int64_t t = 0; t < n; ++t) {
    uint64_t term = from_i64(coef[t]);
    for (int v = 0; v < nv; ++v) term = mulp(term, spow(point[v], inv[v], exps[t * nv + v]));
    acc = addp(acc, term);
  }
  return acc;
}

// Same with fp64 coefficients, each mapped exactly (a finite double is an
// integer times a power of two).
uint64_t oracle_laurent_eval_modp_f64(int nv, int64_t n, const int32_t* exps, const double* coef,
                                      const uint64_t* point) {
  uint64_t inv[MAXV];
  for (int v = 0; v < nv; ++v) inv[v] = invp(point[v]);
  uint64_t acc = 0;
  for (int64_t t = 0; t < n; ++t) {
    uint64_t term = from_f64(coef[t]);
    for (int v = 0; v < nv; ++v) term = mulp(term, spow(point[v], inv[v], exps[t * nv + v]));
    acc = addp(acc, term);
  }
  return acc;
}

// Poisson series evaluated over F_{p^2}: x_k -> r_k in F_p, and the ring map
// exp(i y_k) -> Z_k, i.e. cos(j.y) -> (Z^j + Z^-j)/2, sin(j.y) -> (Z^j - Z^-j)/(2i).
// Result written as (re, im).
void oracle_poisson_eval_fp2(int nx, int ny, int64_t n, const int32_t* x, const int32_t* y,
                             const uint8_t* is_sin, const double* coef, const uint64_t* xpoint,
                             const uint64_t* zre, const uint64_t* zim, uint64_t* out) {
  uint64_t xinv[MAXV];
  for (int v = 0; v < nx; ++v) xinv[v] = invp(xpoint[v]);
  G z[MAXV], zi[MAXV];
  for (int v = 0; v < ny; ++v) {
    z[v] = G{zre[v], zim[v]};
    zi[v] = ginv(z[v]);
  }
  const uint64_t half = invp(2);
  const G inv2i = ginv(G{0, 2});
  G acc{0, 0};
  for (int64_t t = 0; t < n; ++t) {
    uint64_t c = from_f64(coef[t]);
    for (int v = 0; v < nx; ++v) c = mulp(c, spow(xpoint[v], xinv[v], x[t * nx + v]));
    G zp{1, 0}, zm{1, 0};
    for (int v = 0; v < ny; ++v) {
      int64_t e = y[t * ny + v];
      G a = e >= 0 ? gpow(z[v], e) : gpow(zi[v], -e);
      G b = e >= 0 ? gpow(zi[v], e) : gpow(z[v], -e);
      zp = gmul(zp, a);
      zm = gmul(zm, b);
    }
    G trig = is_sin[t] ? gmul(gsub(zp, zm), inv2i) : gmul(gadd(zp, zm), G{half, 0});
    acc = gadd(acc, gmul(trig, G{c, 0}));
  }
  out[0] = acc.re;
  out[1] = acc.im;
}

uint64_t oracle_modp_mul(uint64_t a, uint64_t b) { return mulp(a % P61, b % P61); }
uint64_t oracle_modp_pow(uint64_t a, uint64_t e) { return powp(a % P61, e); }
void oracle_fp2_mul(const uint64_t* a, const uint64_t* b, uint64_t* out) {
  G r = gmul(G{a[0], a[1]}, G{b[0], b[1]});
  out[0] = r.re;
  out[1] = r.im;
}

int oracle_hardware_threads() { return (int)std::thread::hardware_concurrency(); }

}  // extern "C"
