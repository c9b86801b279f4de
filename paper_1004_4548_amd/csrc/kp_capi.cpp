// kp_capi.cpp -- the extern "C" boundary: argument checks, layout and
// workspace planning, mode choice, and the launch sequences of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <climits>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "kp_internal.h"

struct kp_ctx {
  int device = 0;
  int num_cu = 256;
  kp_tune tune{};
  kp::CtxStatus* status = nullptr;   // device
  std::string err;
  bool timing = false;
  bool hash_stats = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;   // pool
  size_t events_used = 0;
  kp::Mailbox* mb = nullptr;          // pinned host-coherent mailbox (host address)
  kp::Mailbox* mb_dev = nullptr;      // the same, device address
  uint64_t seq = 0;                   // last sequence number handed to a kernel
  std::mutex mb_mu;                   // serialises mailbox users
  bool trunc_on = false;              // truncation of Laurent products by weighted degree
  kp::TruncSpec trunc{};
  bool harm_on = false;               // truncation of Poisson products by harmonic order
  kp::HarmonicSpec harm{};
  void* scratch = nullptr;            // device address of this device's scratch array
  hipError_t scratch_err = hipSuccess;
};

namespace kp {

namespace {

constexpr int64_t CODE_LIMIT = (int64_t)1 << 62;
constexpr size_t ALIGN = 256;
constexpr uint64_t GOLDEN_ODD = 0x9E3779B97F4A7C15ull;   // 2^64 / golden ratio, odd

// Workspace of kp_mul_laurent_noalloc: one array per GPU, reserved when this
// code object is loaded on the GPU and kept until the process ends.  Host
// code never uses the name itself (on the host it is only a stand-in for the
// symbol): the device address of each GPU's copy is looked up once per
// device, with that device current, and kept in scratch_ptr.
__device__ __align__(256) unsigned char scratch[KP_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES];
hipError_t scratch_err[MAX_DEVICES];
bool scratch_done[MAX_DEVICES];

// Device address of `device`'s scratch array (the device must be current).
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(scratch_mu);
  if (!scratch_done[device]) {
    void* ptr = nullptr;
    scratch_err[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    scratch_ptr[device] = scratch_err[device] == hipSuccess ? ptr : nullptr;
    scratch_done[device] = true;
  }
  *out = scratch_ptr[device];
  return scratch_err[device];
}

size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

kp_status fail(kp_ctx* ctx, kp_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
kp_status fail(kp_ctx* ctx, kp_status s, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return s;
}

kp_status hip_fail(kp_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, KP_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

// Saturating product of non-negative values.
int64_t sat_mul(int64_t a, int64_t b) {
  int64_t r;
  if (__builtin_mul_overflow(a, b, &r)) return INT64_MAX;
  return r;
}

// Synchronise, read and clear the context's latched device status.
kp_status sync_status(kp_ctx* ctx, hipStream_t s) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  uint32_t bits = 0;
  e = hipMemcpy(&bits, &ctx->status->err, sizeof bits, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(status)");
  if (bits) {
    uint32_t zero = 0;
    e = hipMemcpy(&ctx->status->err, &zero, sizeof zero, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(status clear)");
    kp_status st = (kp_status)first_error(bits);
    return fail(ctx, st, "device reported %s (bits 0x%x)", kp_status_str(st), bits);
  }
  return KP_OK;
}

// Next event pair for timing the accumulation kernel (null when disabled).
std::pair<hipEvent_t, hipEvent_t> timing_pair(kp_ctx* ctx) {
  if (!ctx->timing) return {nullptr, nullptr};
  if (ctx->events_used == ctx->events.size()) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return {nullptr, nullptr};
    ctx->events.emplace_back(a, b);
  }
  return ctx->events[ctx->events_used++];
}

// Device counters {insertions, extra probe steps} when statistics are on.
unsigned long long* hash_stats_ptr(kp_ctx* ctx) {
  return ctx->hash_stats ? &ctx->status->inserts : nullptr;
}

// Words of one array's box as returned by read_boxes: mins, then maxes.
constexpr int BOX_SET = 2 * KP_MAX_VARS;

// Spins until a mailbox word's high half equals `tag` (the low half of the
// call's sequence number, which the kernel side writes above the payload).
// Every few hundred polls the stream is queried, so that a stream that
// failed, or finished without signalling, ends the wait with an error.
kp_status wait_tag(kp_ctx* ctx, const uint64_t* slot, uint64_t tag, hipStream_t s,
                   const char* what) {
  for (uint64_t spins = 1;; ++spins) {
    if ((__atomic_load_n(slot, __ATOMIC_ACQUIRE) >> 32) == tag) return KP_OK;
    __builtin_ia32_pause();
    if ((spins & 255) == 0) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipSuccess) {
        if ((__atomic_load_n(slot, __ATOMIC_ACQUIRE) >> 32) == tag) return KP_OK;
        return fail(ctx, KP_E_DEVICE, "%s: the stream finished without signalling", what);
      }
      if (q != hipErrorNotReady) return hip_fail(ctx, q, what);
    }
  }
}

// The next sequence number (the caller holds mb_mu).  Its low half tags the
// mailbox words and is never 0, the value of a word no kernel has written.
uint64_t bump_seq(kp_ctx* ctx) {
  if ((uint32_t)++ctx->seq == 0) ++ctx->seq;
  return ctx->seq;
}

uint64_t next_seq(kp_ctx* ctx) {
  std::lock_guard<std::mutex> guard(ctx->mb_mu);
  return bump_seq(ctx);
}

// Blocking end of a from-exponents multiply: the count and the latched
// status come back through the mailbox (posted by a kernel already queued
// under `posted`, or else by a post queued here); an error is then read and
// cleared from the status block as by kp_ctx_check.
kp_status wait_count(kp_ctx* ctx, const int64_t* out_n, int64_t* n_host, hipStream_t s,
                     const char* what, uint64_t posted = 0) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, what);
  int64_t n;
  uint32_t err;
  {
    const uint64_t seq = posted ? posted : next_seq(ctx);
    std::lock_guard<std::mutex> guard(ctx->mb_mu);
    if (!posted) {
      e = launch_post_count(out_n, &ctx->status->err, ctx->mb_dev, seq, s);
      if (e != hipSuccess) return hip_fail(ctx, e, what);
    }
    const uint64_t tag = (uint64_t)(uint32_t)seq;
    uint64_t w[3];
    for (int k = 0; k < 3; ++k) {
      kp_status st = wait_tag(ctx, &ctx->mb->n_tag[k], tag, s, what);
      if (st != KP_OK) return st;
      w[k] = __atomic_load_n(&ctx->mb->n_tag[k], __ATOMIC_ACQUIRE) & 0xffffffffu;
    }
    n = (int64_t)(w[0] | (w[1] << 32));
    err = (uint32_t)w[2];
  }
  if (n < 0 || err) {
    kp_status st = sync_status(ctx, s);
    return st != KP_OK ? st : fail(ctx, n < 0 ? (kp_status)(-n) : KP_E_DEVICE, "%s", what);
  }
  if (n_host) *n_host = n;
  return KP_OK;
}

// Per-variable (min, max) of up to four exponent arrays: one launch, the
// result through the mailbox.  res receives, per array, KP_MAX_VARS mins
// then KP_MAX_VARS maxes; an empty array gives min 0 and max -1.
kp_status read_boxes(kp_ctx* ctx, int nseg, const int32_t* const* vals, const int64_t* n,
                     const int32_t* nv, int32_t* res, hipStream_t s) {
  std::lock_guard<std::mutex> guard(ctx->mb_mu);
  BoxArgs A{};
  A.nseg = nseg;
  for (int g = 0; g < nseg; ++g) {
    A.vals[g] = vals[g];
    A.n[g] = n[g];
    A.nv[g] = nv[g];
  }
  A.mb = ctx->mb_dev;
  A.seq = bump_seq(ctx);
  hipError_t e = launch_boxes(A, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "factor boxes");
  // every partial word of this call carries the sequence number's low half
  const uint64_t tag = (uint64_t)(uint32_t)A.seq;
  const int parts = box_parts(A);
  for (int g = 0; g < nseg; ++g) {
    int32_t* r = res + g * BOX_SET;
    for (int v = 0; v < KP_MAX_VARS; ++v) {
      r[v] = INT_MAX;
      r[KP_MAX_VARS + v] = INT_MIN;
    }
    for (int k = 0; k < parts; ++k)
      for (int v = 0; v < nv[g]; ++v)
        for (int side = 0; side < 2; ++side) {
          const uint64_t* slot = &ctx->mb->box_part[g][k][side * KP_MAX_VARS + v];
          kp_status st = wait_tag(ctx, slot, tag, s, "factor boxes");
          if (st != KP_OK) return st;
          const int32_t x = (int32_t)(uint32_t)__atomic_load_n(slot, __ATOMIC_ACQUIRE);
          int32_t& out = r[side * KP_MAX_VARS + v];
          out = side ? std::max(out, x) : std::min(out, x);
        }
    if (n[g] == 0)   // an empty array: min 0, max -1
      for (int v = 0; v < KP_MAX_VARS; ++v) {
        r[v] = 0;
        r[KP_MAX_VARS + v] = -1;
      }
  }
  return KP_OK;
}

// Workspace of the from-exponents entry points: the factors' codes, the
// result's codes, then the multiply's own workspace.
size_t exps_workspace(int poisson, int64_t na, int64_t nb, int64_t max_out, size_t mul_ws) {
  const size_t k = poisson ? 2 : 1;
  return k * align_up(8 * (size_t)na) + k * align_up(8 * (size_t)nb) +
         align_up(8 * (size_t)std::max<int64_t>(max_out, 1)) + mul_ws;
}

kp_status finish(kp_ctx* ctx, unsigned flags, hipStream_t s, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, what);
  if (flags & KP_FLAG_ASYNC) return KP_OK;
  return sync_status(ctx, s);
}

// ------------------------------------------------------------ planning
struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    size_t o = off;
    off = align_up(off + count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

struct Plan {
  kp_mode mode = KP_HASH;
  int64_t max_out = 0;
  size_t ws = 0;
  // dense
  DensePlan dp{};
  // hash
  int64_t cap = 64;
  // partitioned hash: rows of A per workgroup, log2 partitions and bins,
  // count/scatter workgroups, products bound
  bool radix = false;
  int rows = 0, l1 = 1, l2 = 0, blog = 11;   // blog: log2 of a bin's LDS slots
  int64_t nblocks = 0, nprod = 0;
  bool trunc = false;   // truncation tables follow the mode's workspace
  bool harm = false;    // Poisson truncation by harmonic order (term orders in the workspace)
  bool harm_exact = false;   // ... from the factors' multipliers, packed as bytes
  int cw = 1;           // 64-bit words per result coefficient (2 for KP_I128)
  // bucketed table: slots per bucket, buckets, overflow slots, term order
  bool bucket = false;
  int bm = 0;
  int64_t nbuckets = 0, ovcap = 0;
  bool order = false;
  // grouped by code range: ranges of 2^rw codes, row splits of A, bins, B buckets
  bool range = false;
  int rw = 0;
  int64_t rnr = 0, rnsplit = 1, rrows = 0, rbins = 0, rnbk = 0, rsplit_cap = 1;
  int rshift = 0;
  int64_t rtarget = 1;
};

// Truncation tables: slack of A's terms and degree of B's (input order),
// and in dense mode their bucket-sorted copies.
struct TruncBufs {
  int32_t* sa; int32_t* tb;
  int32_t* sa_sorted; int32_t* tb_sorted;
};
void carve_trunc(Carver& c, const Plan& p, int64_t na, int64_t nb, TruncBufs* t) {
  *t = TruncBufs{};
  if (!p.trunc) return;
  t->sa = c.take<int32_t>(na);
  t->tb = c.take<int32_t>(nb);
  if (p.mode == KP_DENSE) {
    t->sa_sorted = c.take<int32_t>(na);
    t->tb_sorted = c.take<int32_t>(nb);
  }
}

int64_t factor_maxcode(const kp_layout* L, int which) {
  int64_t m = 0;
  for (int v = 0; v < L->nx; ++v)
    m += L->xc[v] * (int64_t)(which ? L->bmax[v] - L->bmin[v] : L->amax[v] - L->amin[v]);
  return m;
}

// Work items of a dense product are at most ceil(rows / 64) + 3 per
// (window, tile) pair.  A row of A is visited by a tile in the windows that
// meet an interval of (bucket width of A + tile span + S) codes, at most
// (bwA + span) / S + 2 of them, and the tiles' spans add up to at most
// (buckets of B + tiles) * bucket width of B, B being sorted by bucket.
double dense_items_bound(const DensePlan& d, int64_t na) {
  const double bwA = (double)((int64_t)1 << d.shiftA), bwB = (double)((int64_t)1 << d.shiftB);
  const double nt = (double)d.ntiles, S = (double)d.S;
  double rows = (double)na * ((nt * bwA + ((double)d.nbkB + nt) * bwB) / S + 2.0 * nt);
  rows = std::min(rows, (double)na * nt * (double)d.nwin);
  const double pairs = std::min((double)d.nwin * nt, nt * (((double)d.maxcodeA + bwA) / S + 2.0) +
                                                         ((double)d.nbkB + nt) * bwB / S);
  return rows / DENSE_ITEM_ROWS + 3.0 * pairs + 64.0;
}

// Codes per LDS window: the tuned window for 8-byte slots; 128-bit slots
// take twice the bytes, so half as many codes (a multiple of DENSE_CHUNK).
int64_t dense_window(const kp_ctx* ctx, kp_dtype dt) {
  const int64_t S = ctx->tune.window;
  if (dt != KP_I128) return S;
  return std::max<int64_t>(DENSE_CHUNK, S / 2 / DENSE_CHUNK * DENSE_CHUNK);
}

bool dense_feasible(const kp_ctx* ctx, int64_t S, int64_t nkeys, int64_t na, int64_t nb) {
  if (nkeys > ctx->tune.dense_max_keys || nkeys > DENSE_MAX_CODES) return false;
  if (sat_mul((nkeys + S - 1) / S, (nb + DENSE_TILE - 1) / DENSE_TILE) > ((int64_t)1 << 24))
    return false;
  if (na >= ((int64_t)1 << 31) || nb >= ((int64_t)1 << 29)) return false;
  return true;
}

// Poisson products in dense mode: codes U + s N of the unfolded product in
// eight segments s (piece, type of A, type of B), N = Wx (2 Hy + 1).
struct PoissonDense {
  int64_t N, Hya, Hyb, nkeys, maxA, maxB;
};
PoissonDense poisson_dense_codes(const kp_layout* L) {
  PoissonDense q{};
  int64_t hya = 0, hyb = 0;
  for (int k = 0; k < L->ny; ++k) {
    hya += L->yc[k] * L->ha[k];
    hyb += L->yc[k] * L->hb[k];
  }
  q.Hya = hya;
  q.Hyb = hyb;
  const double N = (double)L->Wx * (2.0 * (double)L->Hy + 1.0);
  if (N * 8.0 > (double)DENSE_MAX_CODES) {
    q.nkeys = INT64_MAX;
    return q;
  }
  q.N = L->Wx * (2 * L->Hy + 1);
  q.nkeys = 8 * q.N;
  q.maxA = 2 * q.N + L->Wx * (2 * hya + 1) - 1;
  q.maxB = 5 * q.N + L->Wx * (2 * hyb + 1) - 1;
  return q;
}

template <bool CARVE>
void carve_dense(Carver& c, const Plan& p, int64_t na, int64_t nb, DenseBufs* B) {
  const DensePlan& d = p.dp;
  Meta* meta = c.take<Meta>(1);
  uint64_t* apk = c.take<uint64_t>(na);
  uint64_t* ac = c.take<uint64_t>(na);
  uint64_t* bpk = c.take<uint64_t>(nb);
  uint64_t* bc = c.take<uint64_t>(nb);
  int32_t* rank_a = c.take<int32_t>(na);
  int32_t* rank_b = c.take<int32_t>(nb);
  int32_t* bstart = c.take<int32_t>(d.nbkA + 1);
  int32_t* bstartB = c.take<int32_t>(d.nbkB + 1);
  int64_t* tmin = c.take<int64_t>(d.ntiles);
  int64_t* tmax = c.take<int64_t>(d.ntiles);
  int64_t* win = c.take<int64_t>(5 * (d.nwin + 1));
  int4* recs = c.take<int4>(d.nwin * d.ntiles);
  uint64_t* items = c.take<uint64_t>(d.items_cap);
  int32_t* task_w = c.take<int32_t>(d.max_tasks);
  int32_t* task_begin = c.take<int32_t>(d.max_tasks + 1);
  int64_t* dense = c.take<int64_t>(d.nwin * d.S * p.cw);
  int64_t* stage_k = c.take<int64_t>(d.nchunk * DENSE_CHUNK);
  int64_t* stage_c = c.take<int64_t>(d.nchunk * DENSE_CHUNK * p.cw);
  int64_t* ccount = c.take<int64_t>(d.nchunk);
  int64_t* coff = c.take<int64_t>(d.nchunk);
  if (CARVE) {
    B->meta = meta;
    B->apk = apk;
    B->ac = ac;
    B->bpk = bpk;
    B->bc = bc;
    B->rank_a = rank_a;
    B->rank_b = rank_b;
    B->bstart = bstart;
    B->bstartB = bstartB;
    B->tmin = tmin;
    B->tmax = tmax;
    B->win = win;
    B->recs = recs;
    B->items = items;
    B->task_w = task_w;
    B->task_begin = task_begin;
    B->dense = dense;
    B->stage_k = stage_k;
    B->stage_c = stage_c;
    B->ccount = ccount;
    B->coff = coff;
    B->na = na;
    B->nb = nb;
  }
}

struct PoissonDenseBufs {
  int64_t* a_codes;
  double* a_coef;
  int64_t* b_codes;
  double* b_coef;
};

template <bool CARVE>
void carve_poisson_dense(Carver& c, int64_t na, int64_t nb, PoissonDenseBufs* q) {
  int64_t* ak = c.take<int64_t>(na);
  double* ac = c.take<double>(na);
  int64_t* bk = c.take<int64_t>(2 * nb);
  double* bc = c.take<double>(2 * nb);
  if (CARVE) *q = PoissonDenseBufs{ak, ac, bk, bc};
}

struct RangeCarve {
  int64_t* bk; uint64_t* bc; int32_t* b_tb; int32_t* brank; int32_t* bstart;
  int64_t* rcount; int32_t* rnb; int64_t* rbin0; int64_t* rtotal; int64_t* rbase;
  int64_t* rhole; int64_t* rabove; int64_t* cnt; int32_t* rns; int64_t* rupre; int64_t* rcbase;
  int32_t* umap;
  int32_t* bin_range; int64_t* bin_start; int64_t* bin_terms; int64_t* bhole; int64_t* babove;
  void* ent;
};

struct HashCarve {
  Meta* meta;
  RangeCarve rg;
  uint64_t* table;
  // bucketed table with its term order: both factors reordered, rank scratch
  int64_t* ord_ak; uint64_t* ord_ac; int64_t* ord_bk; uint64_t* ord_bc;
  int32_t* ord_rank; int32_t* ord_sa; int32_t* ord_tb;
  PoissonPrep pp;
  uint32_t* counts;
  int64_t* pstart;
  int64_t* bstart;
  uint4* ent1;
  uint4* ent2;
  uint16_t* bin1;
};

// Shape of the partitioned accumulation: at most half a bin's LDS table of
// products per bin on average, at most 2^10 partitions and 2^10 bins each;
// about 4096 count/scatter workgroups.
void radix_shape(int64_t na, int64_t nb, int64_t nprod, int bin_slots, Plan* p) {
  p->blog = bin_slots == 8192 ? 13 : bin_slots == 4096 ? 12 : 11;
  int bits = 1;
  while (bits < 20 && ((int64_t)bin_slots / 2 << bits) < nprod) ++bits;
  p->l2 = std::min(10, bits / 2);
  p->l1 = std::max(1, bits - p->l2);
  const int64_t bx = std::max<int64_t>(1, (nb + RADIX_THREADS - 1) / RADIX_THREADS);
  int64_t rows = (na * bx + 4095) / 4096;
  rows = std::max<int64_t>(rows, (na + 65534) / 65535);   // grid.y limit
  p->rows = (int)std::max<int64_t>(1, std::min<int64_t>(rows, (int64_t)1 << 30));
  p->nblocks = bx * std::max<int64_t>(1, (na + p->rows - 1) / p->rows);
  p->nprod = std::max<int64_t>(nprod, 1);
}

// Shape of the accumulation grouped by code range: about 2^18 products per
// range (at least 256 ranges, at most 16384, never more than codes), enough
// row splits of A for about 2048 counting workgroups, bins of half a table,
// and B's buckets (about two per term, as for dense mode).
void range_shape(const kp_layout* L, int64_t na, int64_t nb, int64_t nprod, int bin_slots,
                 int max_bin_bits, int fill, Plan* p) {
  int K = 0;
  while (K < 62 && ((int64_t)1 << K) < L->nkeys) ++K;
  int lr = 8;
  while (lr < 14 && ((int64_t)1 << (lr + 18)) < nprod) ++lr;
  lr = std::min(lr, K);
  p->rw = K - lr;
  p->rnr = std::max<int64_t>(1, (L->nkeys + ((int64_t)1 << p->rw) - 1) >> p->rw);
  p->rnsplit = std::max<int64_t>(1, std::min<int64_t>(16, (2048 + p->rnr - 1) / p->rnr));
  p->rnsplit = std::min<int64_t>(p->rnsplit, std::max<int64_t>(1, na));
  p->rrows = (na + p->rnsplit - 1) / p->rnsplit;
  // a range may take up to four times the even share of splits (the device
  // gives each range splits in proportion to its products)
  p->rsplit_cap = std::max<int64_t>(1, std::min<int64_t>({64, 4 * p->rnsplit, na}));
  p->blog = bin_slots == 8192 ? 13 : bin_slots == 4096 ? 12 : 11;
  // products per bin: `fill` percent of the table's slots (the bound on
  // products exceeds them by a few percent), so that linear probing stays short
  p->rtarget = std::max<int64_t>(1, ((int64_t)fill << p->blog) / 100);
  p->nprod = std::max<int64_t>(nprod, 1);
  // bins: at most two per 2^rtarget products (bucket granularity adds a few
  // candidates per row and range) plus one per range
  // (a range's bins are its bound on products over rtarget, rounded up; the
  // bound exceeds the products by a few terms of B per row and range)
  const double cand = (double)nprod + (double)na * (double)p->rnr;
  const int bb = std::max(0, std::min(10, max_bin_bits));
  p->rbins = std::min<int64_t>(p->rnr << bb,
                               p->rnr + (int64_t)std::ceil(cand / (double)p->rtarget));
  p->rbins = std::max<int64_t>(p->rbins, p->rnr);
  const int64_t maxB = factor_maxcode(L, 1);
  p->rshift = dense_bucket_shift(maxB, nb);
  p->rnbk = (maxB >> p->rshift) + 1;
}

void carve_hash(Carver& c, const Plan& p, int poisson, int64_t na, int64_t nb, HashCarve* h) {
  h->meta = c.take<Meta>(1);
  h->table = nullptr;
  h->counts = nullptr;
  h->pstart = h->bstart = nullptr;
  h->ent1 = h->ent2 = nullptr;
  h->bin1 = nullptr;
  h->ord_ak = h->ord_bk = nullptr;
  h->ord_ac = h->ord_bc = nullptr;
  h->ord_rank = h->ord_sa = h->ord_tb = nullptr;
  h->rg = RangeCarve{};
  if (p.range) {
    RangeCarve& g = h->rg;
    g.bk = c.take<int64_t>(nb);
    g.bc = c.take<uint64_t>(nb);
    g.b_tb = p.trunc ? c.take<int32_t>(nb) : nullptr;
    g.brank = c.take<int32_t>(nb);
    g.bstart = c.take<int32_t>(p.rnbk + 1);
    g.rcount = c.take<int64_t>(p.rnr);
    g.rnb = c.take<int32_t>(p.rnr);
    g.rbin0 = c.take<int64_t>(p.rnr + 1);
    g.rtotal = c.take<int64_t>(p.rnr);
    g.rbase = c.take<int64_t>(p.rnr);
    g.rhole = c.take<int64_t>(p.rnr + 1);
    g.rabove = c.take<int64_t>(p.rnr + 1);
    g.cnt = c.take<int64_t>((size_t)(p.rbins * p.rsplit_cap));
    g.rns = c.take<int32_t>(p.rnr);
    g.rupre = c.take<int64_t>(p.rnr + 1);
    g.rcbase = c.take<int64_t>(p.rnr + 1);
    g.umap = c.take<int32_t>((size_t)(p.rnr * p.rsplit_cap));
    g.bin_range = c.take<int32_t>(p.rbins);
    g.bin_start = c.take<int64_t>(p.rbins + 1);
    g.bin_terms = c.take<int64_t>(p.rbins);
    g.bhole = c.take<int64_t>(p.rbins);
    g.babove = c.take<int64_t>(p.rbins);
    g.ent = c.take<uint4>((size_t)p.nprod);
  } else if (p.radix) {
    const int64_t P1 = (int64_t)1 << p.l1, bins = P1 << p.l2;
    h->counts = c.take<uint32_t>((size_t)(P1 * p.nblocks));
    h->pstart = c.take<int64_t>((size_t)P1 + 1);
    h->bstart = c.take<int64_t>((size_t)bins + 1);
    h->ent1 = c.take<uint4>((size_t)p.nprod);
    h->ent2 = c.take<uint4>((size_t)p.nprod);
    h->bin1 = c.take<uint16_t>((size_t)p.nprod);
  } else {
    const int64_t slots = p.bucket ? p.nbuckets * p.bm + p.ovcap : p.cap;
    h->table = c.take<uint64_t>((size_t)(p.cw == 2 ? 4 : 2) * slots);   // 16- or 32-byte slots
    if (p.bucket && p.order) {
      h->ord_ak = c.take<int64_t>(na);
      h->ord_ac = c.take<uint64_t>(na);
      h->ord_bk = c.take<int64_t>(nb);
      h->ord_bc = c.take<uint64_t>(nb);
      h->ord_rank = c.take<int32_t>(na + nb);
      if (p.trunc) {
        h->ord_sa = c.take<int32_t>(na);
        h->ord_tb = c.take<int32_t>(nb);
      }
    }
  }
  h->pp = PoissonPrep{};
  if (poisson) {
    h->pp.ap = c.take<int64_t>(na);
    h->pp.akx = c.take<int64_t>(na);
    h->pp.at = c.take<uint8_t>(na);
    h->pp.bp = c.take<int64_t>(nb);
    h->pp.bm = c.take<int64_t>(nb);
    h->pp.bkx = c.take<int64_t>(nb);
    h->pp.bt = c.take<uint8_t>(nb);
    if (p.harm_exact) {
      h->pp.ad = c.take<uint4>(na);
      h->pp.bd = c.take<uint4>(nb);
    } else if (p.harm) {
      h->pp.ao = c.take<int32_t>(na);
      h->pp.bo = c.take<int32_t>(nb);
    }
  }
}

kp_status make_plan(kp_ctx* ctx, const kp_layout* L, int poisson, kp_dtype dt, kp_mode mode,
                    int64_t na, int64_t nb, Plan* p) {
  if (!L) return fail(ctx, KP_E_ARG, "null layout");
  if (na < 0 || nb < 0) return fail(ctx, KP_E_ARG, "negative factor size");
  if (dt != KP_I64 && dt != KP_F64 && dt != KP_I128)
    return fail(ctx, KP_E_ARG, "bad dtype %d", (int)dt);
  if (poisson && dt != KP_F64)
    return fail(ctx, KP_E_DTYPE, "Poisson products carry a factor 1/2 and need fp64 coefficients");
  if (mode != KP_AUTO && mode != KP_DENSE && mode != KP_HASH)
    return fail(ctx, KP_E_ARG, "bad mode %d", (int)mode);
  if (L->nkeys < 0 || L->nkeys >= CODE_LIMIT) return fail(ctx, KP_E_CODE_OVERFLOW, "key space");
  int64_t pairs = sat_mul(na, nb);
  int64_t contrib = poisson ? sat_mul(pairs, 2) : pairs;
  p->max_out = std::min(contrib, L->nkeys);
  // dense mode works on (na, nbd) terms in a space of dn codes; a Poisson
  // product's B appears twice (difference and sum pieces)
  const PoissonDense pq = poisson ? poisson_dense_codes(L) : PoissonDense{};
  const int64_t dn = poisson ? pq.nkeys : L->nkeys;
  const int64_t nbd = poisson ? sat_mul(nb, 2) : nb;
  p->cw = coef_words(dt);
  const int64_t S = dense_window(ctx, dt);
  bool dense_ok = dense_feasible(ctx, S, dn, na, nbd);
  if (dense_ok) {
    DensePlan& d = p->dp;
    d.S = S;
    d.nkeys = dn;
    d.nwin = std::max<int64_t>(1, (dn + d.S - 1) / d.S);
    d.nchunk = std::max<int64_t>(1, (dn + DENSE_CHUNK - 1) / DENSE_CHUNK);
    d.ntiles = std::max<int64_t>(1, (nbd + DENSE_TILE - 1) / DENSE_TILE);
    d.block = ctx->tune.block;
    d.target_tasks = std::max<int64_t>(1, (int64_t)ctx->num_cu * ctx->tune.tasks_per_cu);
    d.max_tasks = d.target_tasks;
    d.min_work = 512;
    d.maxcodeA = poisson ? pq.maxA : factor_maxcode(L, 0);
    d.maxcodeB = poisson ? pq.maxB : factor_maxcode(L, 1);
    d.accumulate = poisson ? 1 : 0;
    d.shiftA = dense_bucket_shift(d.maxcodeA, na);
    d.shiftB = dense_bucket_shift(d.maxcodeB, nbd);
    d.nbkA = (d.maxcodeA >> d.shiftA) + 1;
    d.nbkB = (d.maxcodeB >> d.shiftB) + 1;
    const double items = dense_items_bound(d, na);
    dense_ok = items <= (double)((int64_t)1 << 31);
    d.items_cap = dense_ok ? (int64_t)items : 0;
  }
  kp_mode m = mode;
  const bool harm = poisson && ctx->harm_on;
  if (harm && m == KP_DENSE)
    return fail(ctx, KP_E_MODE, "a Poisson product truncated by harmonic order runs in hash mode");
  if (m == KP_AUTO) {
    double budget = ctx->tune.dense_keys_per_pair * (double)contrib;
    m = (!harm && dense_ok && (double)dn <= budget) ? KP_DENSE : KP_HASH;
  }
  if (m == KP_DENSE && !dense_ok)
    return fail(ctx, KP_E_MODE,
                "dense mode needs a product with at most %lld codes and a bounded "
                "number of work items",
                (long long)std::min<int64_t>(ctx->tune.dense_max_keys, DENSE_MAX_CODES));
  p->mode = m;
  p->trunc = ctx->trunc_on && !poisson;
  p->harm = harm;
  if (harm) {   // every factor multiplier fits a signed byte: exact orders per piece
    bool small = true;
    for (int v = 0; v < L->ny; ++v) small = small && L->ha[v] <= 127 && L->hb[v] <= 127;
    p->harm_exact = small;
  }
  Carver c;
  if (m == KP_DENSE) {
    carve_dense<false>(c, *p, na, nbd, nullptr);
    if (poisson) carve_poisson_dense<false>(c, na, nb, nullptr);
  } else {
    int64_t want;
    if (ctx->tune.hash_capacity > 0) {
      want = ctx->tune.hash_capacity;
    } else {
      double w = (double)std::max<int64_t>(p->max_out, 1) / ctx->tune.hash_load;
      want = w > 4.0e18 ? INT64_MAX : (int64_t)w + 1;
    }
    p->cap = std::max<int64_t>(64, want);
    if (p->cap > ((int64_t)1 << 40))
      return fail(ctx, KP_E_CAPACITY, "hash table would need %lld slots", (long long)p->cap);
    // partitioned when asked for, or (auto) when the products are not many
    // more than the result bound: its workspace is 32 bytes per product
    // against 32 per result slot pair of the global table
    // the paper's bucketed table when asked for (Laurent, 8-byte coefficients)
    p->bucket = ctx->tune.hash_bucket > 0 && !poisson && dt != KP_I128;
    if (p->bucket) {
      p->bm = ctx->tune.hash_bucket;
      p->nbuckets = (p->cap + p->bm - 1) / p->bm;
      // overflow table: six times the codes expected to overflow when the
      // bound's codes spread over the buckets as a Poisson variable X of mean
      // lam, N E[(X - m)+]: the highly sparse benchmark product (m = 8, load
      // 0.5) overflowed 2.5 times the estimate, which leaves the table 40 % full
      const double lam = (double)std::max<int64_t>(p->max_out, 1) / (double)p->nbuckets;
      double pk = std::exp(-lam), below = 0.0;
      for (int k = 0; k <= p->bm; ++k) {
        below += (double)(p->bm - k) * pk;
        pk *= lam / (double)(k + 1);
      }
      const double excess = std::max(0.0, lam - (double)p->bm + below);
      p->ovcap = std::max<int64_t>(1024, (int64_t)std::ceil(6.0 * excess * (double)p->nbuckets));
      p->order = ctx->tune.hash_order != 0;
    }
    // (128-bit sums: the grouped entries carry 32-bit term indices, and the
    // bins' LDS tables of 24-byte slots hold at most 4096)
    const bool idx32 = na < ((int64_t)1 << 32) && nb < ((int64_t)1 << 32);
    // (a harmonic truncation always takes the grouped layout, whose bins
    // drop the terms over the limit)
    p->radix = !p->bucket && (dt != KP_I128 || idx32) &&
               (harm || ctx->tune.hash_partitioned == 2 ||
                (ctx->tune.hash_partitioned == 1 &&
                 (double)contrib <= 4.0 * (double)std::max<int64_t>(p->max_out, 1)));
    // (a wavefront scans the interval lengths of 64 rows in 32 bits)
    // Automatic grouping: by ranges for products spread thinly over the code
    // space (at most one product per 64 codes: most are distinct terms, and
    // each is written once), else two levels of hash bits, which also take a
    // truncated product (they drop a pair over the limit before forming it,
    // while the ranges enumerate every pair of a row's interval of B).
    const int grouping = ctx->tune.hash_grouping;
    const bool thin = (double)contrib * 64.0 <= (double)L->nkeys;
    p->range = p->radix && !poisson && dt != KP_I128 &&
               (grouping == 2 || (grouping == 0 && !p->trunc && thin)) &&
               na < ((int64_t)1 << 31) && nb <= ((int64_t)1 << 24);
    if (p->range) {
      p->radix = false;
      range_shape(L, na, nb, contrib, ctx->tune.hash_bin_slots, ctx->tune.hash_max_bin_bits,
                  ctx->tune.hash_bin_fill, p);
    }
    if (p->radix) {
      if (contrib > ((int64_t)1 << 36))
        return fail(ctx, KP_E_CAPACITY, "%lld products exceed the partitioned table",
                    (long long)contrib);
      const int slots = dt == KP_I128 ? std::min(ctx->tune.hash_bin_slots, 4096)
                                      : ctx->tune.hash_bin_slots;
      radix_shape(na, nb, contrib, slots, p);
    }
    HashCarve h;
    carve_hash(c, *p, poisson, na, nb, &h);
  }
  TruncBufs tb;
  carve_trunc(c, *p, na, nb, &tb);
  p->ws = c.off;
  return KP_OK;
}

}  // namespace

DevLayout make_dev_layout(const kp_layout& L, int which) {
  DevLayout d{};
  d.nx = L.nx;
  d.ny = L.ny;
  d.Wx = L.Wx;
  d.Hy = L.Hy;
  d.nkeys = L.nkeys;
  for (int v = 0; v < L.nx; ++v) {
    d.fmin[v] = which ? L.bmin[v] : L.amin[v];
    d.fmax[v] = which ? L.bmax[v] : L.amax[v];
    d.xc[v] = L.xc[v];
    d.xmin[v] = L.xmin[v];
    d.dx[v] = make_fastdiv((uint64_t)L.xw[v]);
    d.dx32[v] = make_fastdiv32((uint64_t)L.xw[v]);
  }
  for (int v = 0; v < L.ny; ++v) {
    d.fh[v] = which ? L.hb[v] : L.ha[v];
    d.yc[v] = L.yc[v];
    d.yh[v] = L.yh[v];
    d.dy[v] = make_fastdiv((uint64_t)(2 * L.yh[v] + 1));
  }
  d.dWx = make_fastdiv((uint64_t)std::max<int64_t>(L.Wx, 1));
  return d;
}

}  // namespace kp

using namespace kp;

extern "C" {

const char* kp_status_str(kp_status s) {
  switch (s) {
    case KP_OK: return "ok";
    case KP_E_ARG: return "invalid argument";
    case KP_E_RANGE: return "exponent outside the layout box";
    case KP_E_CODE_OVERFLOW: return "product box exceeds the 62-bit code space";
    case KP_E_NONCANONICAL: return "Poisson term not in canonical form";
    case KP_E_CAPACITY: return "output or table capacity too small";
    case KP_E_WORKSPACE: return "workspace too small";
    case KP_E_DEVICE: return "HIP runtime error";
    case KP_E_DTYPE: return "coefficient type not supported";
    case KP_E_MODE: return "accumulator mode not possible for this layout";
  }
  return "unknown status";
}

const char* kp_last_error(const kp_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

kp_status kp_ctx_create(int device, kp_ctx** out) {
  if (!out) return KP_E_ARG;
  *out = nullptr;
  auto* ctx = new kp_ctx;
  ctx->device = device;
  ctx->tune.window = 18432;
  ctx->tune.block = 1024;
  ctx->tune.tasks_per_cu = 1;
  ctx->tune.hash_load = 0.5;
  ctx->tune.hash_capacity = 0;
  ctx->tune.dense_max_keys = (int64_t)1 << 27;
  ctx->tune.dense_keys_per_pair = 8.0;
  ctx->tune.hash_rows = 64;
  ctx->tune.hash_partitioned = 1;
  ctx->tune.hash_bucket = 0;
  ctx->tune.hash_order = 1;
  ctx->tune.hash_bin_slots = 4096;
  ctx->tune.hash_grouping = 0;
  ctx->tune.hash_max_bin_bits = 10;
  ctx->tune.hash_bin_fill = 42;
  if (device < 0) {   // host-only context: planning (kp_mul_bound) and tuning only
    *out = ctx;
    return KP_OK;
  }
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return KP_E_DEVICE;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cus > 0)
    ctx->num_cu = cus;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&ctx->status), sizeof(CtxStatus));
  if (e == hipSuccess) e = hipMemset(ctx->status, 0, sizeof(CtxStatus));
  if (e == hipSuccess) e = dense_setup();
  if (e == hipSuccess) e = range_setup();
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&ctx->mb), sizeof(Mailbox),
                      hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) {
    std::memset(ctx->mb, 0, sizeof(Mailbox));
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&ctx->mb_dev), ctx->mb, 0);
  }
  // the allocation-free entry point's workspace (a failure is reported by
  // that entry point, not here)
  if (e == hipSuccess) ctx->scratch_err = scratch_address(device, &ctx->scratch);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    kp_ctx_destroy(ctx);
    return KP_E_DEVICE;
  }
  *out = ctx;
  return KP_OK;
}

kp_status kp_ctx_timing(kp_ctx* ctx, int enable) {
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  ctx->timing = enable != 0;
  return KP_OK;
}

kp_status kp_ctx_timing_read(kp_ctx* ctx, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return KP_E_ARG;
  double tot = 0;
  for (size_t i = 0; i < ctx->events_used; ++i) {
    hipError_t e = hipEventSynchronize(ctx->events[i].second);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->events[i].first, ctx->events[i].second);
    if (e != hipSuccess) {
      ctx->events_used = 0;
      return hip_fail(ctx, e, "kp_ctx_timing_read");
    }
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)ctx->events_used;
  ctx->events_used = 0;
  return KP_OK;
}

kp_status kp_ctx_set_truncation(kp_ctx* ctx, int32_t nvars, const int32_t* weights,
                                int64_t max_degree) {
  if (!ctx) return KP_E_ARG;
  if (nvars < 1 || nvars > KP_MAX_VARS || !weights)
    return fail(ctx, KP_E_ARG, "kp_ctx_set_truncation: 1..%d weights", KP_MAX_VARS);
  TruncSpec t{};
  for (int v = 0; v < nvars; ++v) {
    if (weights[v] < -(1 << 15) || weights[v] > (1 << 15))
      return fail(ctx, KP_E_ARG, "kp_ctx_set_truncation: weights must lie in [-2^15, 2^15]");
    t.w[v] = weights[v];
  }
  t.max_degree = max_degree;
  ctx->trunc = t;
  ctx->trunc_on = true;
  return KP_OK;
}

kp_status kp_ctx_set_harmonic_truncation(kp_ctx* ctx, int32_t ny, const int32_t* weights,
                                         int64_t max_order) {
  using namespace kp;
  if (!ctx) return KP_E_ARG;
  if (ny < 1 || ny > KP_MAX_VARS || !weights)
    return fail(ctx, KP_E_ARG, "kp_ctx_set_harmonic_truncation: 1..%d weights", KP_MAX_VARS);
  HarmonicSpec h{};
  for (int v = 0; v < ny; ++v) {
    if (weights[v] < 0 || weights[v] > (1 << 15))
      return fail(ctx, KP_E_ARG, "kp_ctx_set_harmonic_truncation: weights must lie in [0, 2^15]");
    h.w[v] = weights[v];
  }
  h.max_order = max_order;
  ctx->harm = h;
  ctx->harm_on = true;
  return KP_OK;
}

kp_status kp_ctx_clear_truncation(kp_ctx* ctx) {
  if (!ctx) return KP_E_ARG;
  ctx->trunc_on = false;
  ctx->harm_on = false;
  return KP_OK;
}

kp_status kp_ctx_hash_stats(kp_ctx* ctx, int enable) {
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  ctx->hash_stats = enable != 0;
  return KP_OK;
}

kp_status kp_ctx_hash_stats_read(kp_ctx* ctx, hipStream_t stream, int64_t* inserts,
                                 int64_t* extra_probes, int64_t* overflows) {
  if (!ctx || !inserts || !extra_probes) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  hipError_t e = hipStreamSynchronize(stream);
  unsigned long long v[3] = {0, 0, 0};   // inserts, probes, overflows (consecutive)
  if (e == hipSuccess) e = hipMemcpy(v, &ctx->status->inserts, sizeof v, hipMemcpyDeviceToHost);
  const unsigned long long zero[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpy(&ctx->status->inserts, zero, sizeof zero, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_ctx_hash_stats_read");
  *inserts = (int64_t)v[0];
  *extra_probes = (int64_t)v[1];
  if (overflows) *overflows = (int64_t)v[2];
  return KP_OK;
}

kp_status kp_probe_lds_atomic(kp_ctx* ctx, int pattern, double* adds_per_second,
                              hipStream_t stream) {
  if (!ctx || !adds_per_second) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (pattern < 0 || pattern > 4) return fail(ctx, KP_E_ARG, "pattern must be 0 to 4");
  const int blocks = 2 * ctx->num_cu, iters = 1024;
  float ms = 0;
  hipError_t e = probe_lds_atomic(pattern, blocks, iters, ctx->status->sink, &ms, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_probe_lds_atomic");
  if (!(ms > 0)) return fail(ctx, KP_E_DEVICE, "kp_probe_lds_atomic: no elapsed time");
  *adds_per_second = (double)blocks * 1024.0 * 16.0 * iters / (ms * 1e-3);
  return KP_OK;
}

kp_status kp_ctx_destroy(kp_ctx* ctx) {
  if (!ctx) return KP_E_ARG;
  for (auto& pr : ctx->events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  if (ctx->status) (void)hipFree(ctx->status);
  if (ctx->mb) (void)hipHostFree(ctx->mb);
  delete ctx;
  return KP_OK;
}

kp_status kp_ctx_get_tune(const kp_ctx* ctx, kp_tune* out) {
  if (!ctx || !out) return KP_E_ARG;
  *out = ctx->tune;
  return KP_OK;
}

kp_status kp_ctx_set_tune(kp_ctx* ctx, const kp_tune* t) {
  if (!ctx || !t) return KP_E_ARG;
  if (t->block != 256 && t->block != 512 && t->block != 1024)
    return fail(ctx, KP_E_ARG, "block must be 256, 512 or 1024");
  if (t->window < DENSE_CHUNK || t->window % DENSE_CHUNK != 0 || t->window > DENSE_MAX_WINDOW)
    return fail(ctx, KP_E_ARG, "window must be a multiple of %lld in [%lld, %lld]",
                (long long)DENSE_CHUNK, (long long)DENSE_CHUNK, (long long)DENSE_MAX_WINDOW);
  if (t->tasks_per_cu < 1) return fail(ctx, KP_E_ARG, "tasks_per_cu must be >= 1");
  if (!(t->hash_load >= 0.05 && t->hash_load <= 0.9))
    return fail(ctx, KP_E_ARG, "hash_load must lie in [0.05, 0.9]");
  if (t->dense_max_keys > DENSE_MAX_CODES)
    return fail(ctx, KP_E_ARG, "dense_max_keys must be at most %lld", (long long)DENSE_MAX_CODES);
  if (t->hash_partitioned < 0 || t->hash_partitioned > 2)
    return fail(ctx, KP_E_ARG, "hash_partitioned must be 0, 1 or 2");
  if (t->hash_bucket < 0 || t->hash_bucket > 16)
    return fail(ctx, KP_E_ARG, "hash_bucket must lie in [0, 16]");
  if (t->hash_order != 0 && t->hash_order != 1)
    return fail(ctx, KP_E_ARG, "hash_order must be 0 or 1");
  if (t->hash_bin_slots != 2048 && t->hash_bin_slots != 4096 && t->hash_bin_slots != 8192)
    return fail(ctx, KP_E_ARG, "hash_bin_slots must be 2048, 4096 or 8192");
  if (t->hash_grouping < 0 || t->hash_grouping > 2)
    return fail(ctx, KP_E_ARG, "hash_grouping must be 0, 1 or 2");
  if (t->hash_max_bin_bits < 0 || t->hash_max_bin_bits > 10)
    return fail(ctx, KP_E_ARG, "hash_max_bin_bits must lie in [0, 10]");
  if (t->hash_bin_fill < 10 || t->hash_bin_fill > 90)
    return fail(ctx, KP_E_ARG, "hash_bin_fill must lie in [10, 90]");
  if (t->hash_capacity < 0 || t->dense_max_keys < 0 || t->dense_keys_per_pair < 0 ||
      t->hash_rows < 1)
    return fail(ctx, KP_E_ARG, "negative tuning value");
  ctx->tune = *t;
  return KP_OK;
}

kp_status kp_ctx_check(kp_ctx* ctx, hipStream_t stream) {
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  return sync_status(ctx, stream);
}

kp_status kp_minmax(kp_ctx* ctx, int64_t n, int32_t nvars, const int32_t* vals, int32_t* out,
                    unsigned flags, hipStream_t stream) {
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (n < 0 || nvars < 1 || nvars > KP_MAX_VARS || !out || (n > 0 && !vals))
    return fail(ctx, KP_E_ARG, "kp_minmax: bad arguments");
  hipError_t e = launch_minmax(n, nvars, vals, out, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_minmax");
  return finish(ctx, flags, stream, "kp_minmax");
}

kp_status kp_layout_product(int32_t nx, int32_t ny, const int32_t* amin, const int32_t* amax,
                            const int32_t* bmin, const int32_t* bmax, const int32_t* ha,
                            const int32_t* hb, kp_layout* out) {
  if (!out || nx < 0 || nx > KP_MAX_VARS || ny < 0 || ny > KP_MAX_VARS) return KP_E_ARG;
  if (nx > 0 && (!amin || !amax || !bmin || !bmax)) return KP_E_ARG;
  if (ny > 0 && (!ha || !hb)) return KP_E_ARG;
  kp_layout L;
  std::memset(&L, 0, sizeof L);
  L.nx = nx;
  L.ny = ny;
  bool empty = false;
  int64_t W = 1;
  for (int v = 0; v < nx; ++v) {
    L.amin[v] = amin[v];
    L.amax[v] = amax[v];
    L.bmin[v] = bmin[v];
    L.bmax[v] = bmax[v];
    if (amin[v] > amax[v] || bmin[v] > bmax[v]) {
      empty = true;
      continue;
    }
    L.xmin[v] = (int64_t)amin[v] + bmin[v];
    L.xw[v] = (int64_t)amax[v] + bmax[v] - L.xmin[v] + 1;
    L.xc[v] = W;
    if (__builtin_mul_overflow(W, L.xw[v], &W) || W >= CODE_LIMIT) return KP_E_CODE_OVERFLOW;
  }
  int64_t Wy = 1;
  for (int v = 0; v < ny; ++v) {
    L.ha[v] = ha[v];
    L.hb[v] = hb[v];
    if (ha[v] < 0 || hb[v] < 0) {
      empty = true;
      continue;
    }
    L.yh[v] = (int64_t)ha[v] + hb[v];
  }
  for (int v = ny - 1; v >= 0; --v) {   // y_0 most significant
    if (L.yh[v] < 0) continue;
    L.yc[v] = Wy;
    if (__builtin_mul_overflow(Wy, 2 * L.yh[v] + 1, &Wy) || Wy >= CODE_LIMIT)
      return KP_E_CODE_OVERFLOW;
  }
  L.Wx = W;
  L.Hy = (Wy - 1) / 2;
  if (ny == 0) {
    L.nkeys = W;
  } else {
    int64_t k;
    if (__builtin_mul_overflow(W, L.Hy + 1, &k) || __builtin_mul_overflow(k, (int64_t)2, &k) ||
        k >= CODE_LIMIT)
      return KP_E_CODE_OVERFLOW;
    L.nkeys = k;
  }
  if (empty) L.nkeys = 0;
  *out = L;
  return KP_OK;
}

kp_status kp_encode(kp_ctx* ctx, const kp_layout* layout, int which, int64_t n,
                    const int32_t* x_exps, const int32_t* y_mult, const uint8_t* is_sin,
                    int64_t* xcodes, int64_t* ycodes, unsigned flags, hipStream_t stream) {
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (!layout || (which != 0 && which != 1) || n < 0)
    return fail(ctx, KP_E_ARG, "kp_encode: bad arguments");
  if (n > 0 && ((layout->nx > 0 && !x_exps) || !xcodes ||
                (layout->ny > 0 && (!y_mult || !is_sin || !ycodes))))
    return fail(ctx, KP_E_ARG, "kp_encode: null array");
  DevLayout d = make_dev_layout(*layout, which);
  hipError_t e = launch_encode(d, n, x_exps, y_mult, is_sin, xcodes, ycodes, &ctx->status->err,
                               stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_encode");
  return finish(ctx, flags, stream, "kp_encode");
}

kp_status kp_decode(kp_ctx* ctx, const kp_layout* layout, int poisson, int64_t n,
                    const int64_t* codes, int32_t* x_exps, int32_t* y_mult, uint8_t* is_sin,
                    unsigned flags, hipStream_t stream) {
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (!layout || n < 0) return fail(ctx, KP_E_ARG, "kp_decode: bad arguments");
  if (poisson && layout->ny == 0) return fail(ctx, KP_E_ARG, "kp_decode: layout has no trig part");
  if (n > 0 && (!codes || (layout->nx > 0 && !x_exps) || (poisson && (!y_mult || !is_sin))))
    return fail(ctx, KP_E_ARG, "kp_decode: null array");
  DevLayout d = make_dev_layout(*layout, 0);
  hipError_t e = launch_decode(d, poisson, n, codes, x_exps, y_mult, is_sin, &ctx->status->err,
                               stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_decode");
  return finish(ctx, flags, stream, "kp_decode");
}

kp_status kp_mul_bound(kp_ctx* ctx, const kp_layout* layout, int poisson, kp_dtype dtype,
                       kp_mode mode, int64_t na, int64_t nb, kp_mode* resolved,
                       int64_t* max_out_terms, size_t* workspace_bytes) {
  if (!ctx) return KP_E_ARG;
  Plan p;
  kp_status st = make_plan(ctx, layout, poisson, dtype, mode, na, nb, &p);
  if (st != KP_OK) return st;
  if (resolved) *resolved = p.mode;
  if (max_out_terms) *max_out_terms = p.max_out;
  if (workspace_bytes) *workspace_bytes = p.ws;
  return KP_OK;
}

namespace kp {
namespace {

// Queues one Laurent product (no synchronisation).  `timed`: record the
// context's timing events around the accumulation kernel when enabled.
// Options of the from-exponents path: the multiply writes decoded exponents
// into `exps` (dense: its output copy; partitioned hash: its bins), and the
// dense output scan posts the count to the mailbox under `seq` (0: no post).
// `decoded` and `posted` report which were taken.
struct ExpsOut {
  int32_t* exps;
  DevLayout dec;
  Mailbox* mb;
  uint64_t seq;
  bool decoded;
  bool posted;
};

kp_status enqueue_laurent(kp_ctx* ctx, const kp_layout* layout, kp_dtype dtype, kp_mode mode,
                          const int64_t* a_codes, const void* a_coef, int64_t na,
                          const int64_t* b_codes, const void* b_coef, int64_t nb,
                          int64_t* out_codes, void* out_coef, int64_t out_cap, int64_t* out_n,
                          void* workspace, size_t workspace_bytes, hipStream_t stream,
                          bool timed, ExpsOut* xo = nullptr) {
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  Plan p;
  kp_status st = make_plan(ctx, layout, 0, dtype, mode, na, nb, &p);
  if (st != KP_OK) return st;
  if (!out_n || out_cap < 0 || (na > 0 && (!a_codes || !a_coef)) ||
      (nb > 0 && (!b_codes || !b_coef)) || (out_cap > 0 && (!out_codes || !out_coef)))
    return fail(ctx, KP_E_ARG, "kp_mul_laurent: null array or negative capacity");
  if (workspace_bytes < p.ws || (p.ws > 0 && !workspace))
    return fail(ctx, KP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, p.ws);
  Carver c;
  c.base = static_cast<char*>(workspace);
  hipError_t e = hipSuccess;
  const bool empty = na == 0 || nb == 0 || layout->nkeys == 0;
  // the truncation tables sit after the mode's workspace (as planned)
  TruncBufs tr{};
  {
    Carver t = c;
    if (p.mode == KP_DENSE) {
      carve_dense<false>(t, p, na, nb, nullptr);
    } else {
      HashCarve h;
      carve_hash(t, p, 0, na, nb, &h);
    }
    carve_trunc(t, p, na, nb, &tr);
    if (p.trunc && !empty)
      e = launch_degrees(make_dev_layout(*layout, 0), make_dev_layout(*layout, 1), ctx->trunc, na,
                         nb, a_codes, b_codes, tr.sa, tr.tb, &ctx->status->err, stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "kp_mul_laurent truncation tables");
  }
  if (p.mode == KP_DENSE) {
    DenseBufs B{};
    carve_dense<true>(c, p, na, nb, &B);
    B.a_sa_in = tr.sa;
    B.b_tb_in = tr.tb;
    B.a_sa = tr.sa_sorted;
    B.b_tb = tr.tb_sorted;
    B.a_keys_in = a_codes;
    B.a_coef_in = (const int64_t*)a_coef;
    B.b_keys_in = b_codes;
    B.b_coef_in = (const int64_t*)b_coef;
    B.out_k = out_codes;
    B.out_c = out_coef;
    B.out_cap = out_cap;
    B.out_n = out_n;
    if (xo && !empty) {
      B.out_exps = xo->exps;
      B.dec = xo->dec;
      B.mb = xo->seq ? xo->mb : nullptr;
      B.seq = xo->seq;
      xo->decoded = true;
      xo->posted = xo->seq != 0;
    }
    B.ctx_err = &ctx->status->err;
    if (!empty) {
      if (timed) std::tie(B.ev0, B.ev1) = timing_pair(ctx);
      e = launch_dense_laurent(p.dp, B, dtype, stream);
    } else {
      e = launch_meta_init(B.meta, stream);
      if (e == hipSuccess) e = launch_finalize(B.meta, out_cap, out_n, &ctx->status->err, stream);
    }
  } else {
    HashCarve h;
    carve_hash(c, p, 0, na, nb, &h);
    HashBufs H{h.meta, h.table, p.cap, p.cap, out_codes, out_coef, out_cap,
               nullptr, nullptr, hash_stats_ptr(ctx)};
    H.a_sa = tr.sa;
    H.b_tb = tr.tb;
    if (!empty && timed) std::tie(H.ev0, H.ev1) = timing_pair(ctx);
    e = launch_meta_init(h.meta, stream);
    if (!empty && p.range) {
      const RangeCarve& g = h.rg;
      RangeArgs R{};
      R.meta = h.meta;
      R.ak = a_codes;
      R.ac = a_coef;
      R.na = na;
      R.maxA = factor_maxcode(layout, 0);
      R.bk_in = b_codes;
      R.bc_in = b_coef;
      R.nb = nb;
      R.maxB = factor_maxcode(layout, 1);
      R.a_sa = tr.sa;
      R.b_tb_in = tr.tb;
      R.bk = g.bk;
      R.bc = g.bc;
      R.b_tb = tr.tb ? g.b_tb : nullptr;
      R.brank = g.brank;
      R.bstart = g.bstart;
      R.shiftB = p.rshift;
      R.nbkB = p.rnbk;
      R.nkeys = layout->nkeys;
      R.w = p.rw;
      R.nr = p.rnr;
      // an odd multiplier modulo 2^w and its inverse (Newton's iteration
      // doubles the correct low bits each step: 1, 2, 4, ..., 64)
      const uint64_t m = GOLDEN_ODD;
      uint64_t inv = m;
      for (int k = 0; k < 6; ++k) inv *= 2 - m * inv;
      const uint64_t mask = p.rw >= 64 ? ~0ull : ((1ull << p.rw) - 1);
      R.mult = m & mask;
      R.inv = inv & mask;
      R.nsplit = p.rnsplit;
      R.rows = p.rrows;
      R.split_cap = p.rsplit_cap;
      R.rns = g.rns;
      R.rupre = g.rupre;
      R.rcbase = g.rcbase;
      R.umap = g.umap;
      R.target = p.rtarget;
      R.max_l2 = std::max(0, std::min(10, ctx->tune.hash_max_bin_bits));
      R.nbins_max = p.rbins;
      R.rcount = g.rcount;
      R.rnb = g.rnb;
      R.rbin0 = g.rbin0;
      R.rtotal = g.rtotal;
      R.rbase = g.rbase;
      R.rhole = g.rhole;
      R.rabove = g.rabove;
      R.cnt = g.cnt;
      R.bin_range = g.bin_range;
      R.bin_start = g.bin_start;
      R.bin_terms = g.bin_terms;
      R.bhole = g.bhole;
      R.babove = g.babove;
      R.ent = g.ent;
      R.out_k = out_codes;
      R.out_c = out_coef;
      R.out_cap = out_cap;
      if (xo) {
        R.out_x = xo->exps;
        R.dec = xo->dec;
        xo->decoded = true;
      }
      R.ev0 = H.ev0;
      R.ev1 = H.ev1;
      R.bin_log = p.blog;
      R.stats = H.stats;
      if (e == hipSuccess) e = launch_range(R, dtype, stream);
    } else if (!empty && p.radix) {
      if (e == hipSuccess && dtype == KP_I64)
        e = launch_coef_range((const int64_t*)a_coef, na, (const int64_t*)b_coef, nb, h.meta,
                              stream);
      RadixArgs R{a_codes, a_coef, na, b_codes, b_coef, nb, 0, PoissonPrep{}, p.rows, p.l1,
                  p.l2, 0, h.counts, h.pstart, h.bstart, h.ent1, h.ent2, h.meta, out_codes,
                  out_coef, out_cap, H.stats, H.ev0, H.ev1};
      R.bin_log = p.blog;
      R.bin1 = h.bin1;
      R.a_sa = tr.sa;
      R.b_tb = tr.tb;
      if (xo) {
        R.out_x = xo->exps;
        R.dec = xo->dec;
        xo->decoded = true;
      }
      if (e == hipSuccess)
        e = launch_radix(R, dtype == KP_F64 ? 1 : dtype == KP_I128 ? 3 : 0, stream);
    } else if (!empty) {
      if (e == hipSuccess && dtype == KP_I64)
        e = launch_coef_range((const int64_t*)a_coef, na, (const int64_t*)b_coef, nb, h.meta,
                              stream);
      if (p.bucket) {
        const BucketGeom G{p.bm, (uint64_t)p.nbuckets, make_fastdiv((uint64_t)p.nbuckets),
                           p.ovcap};
        const int64_t* ak = a_codes;
        const int64_t* bk = b_codes;
        const void* ac = a_coef;
        const void* bc = b_coef;
        if (p.order) {   // the terms by code mod N
          ModOrder O{};
          O.k_in[0] = a_codes;
          O.k_in[1] = b_codes;
          O.c_in[0] = static_cast<const uint64_t*>(a_coef);
          O.c_in[1] = static_cast<const uint64_t*>(b_coef);
          O.t_in[0] = p.trunc ? tr.sa : nullptr;
          O.t_in[1] = p.trunc ? tr.tb : nullptr;
          O.n[0] = na;
          O.n[1] = nb;
          O.k_out[0] = h.ord_ak;
          O.k_out[1] = h.ord_bk;
          O.c_out[0] = h.ord_ac;
          O.c_out[1] = h.ord_bc;
          O.t_out[0] = h.ord_sa;
          O.t_out[1] = h.ord_tb;
          O.rank[0] = h.ord_rank;
          O.rank[1] = h.ord_rank + na;
          if (e == hipSuccess) e = launch_mod_order(O, G, stream);
          ak = h.ord_ak;
          bk = h.ord_bk;
          ac = h.ord_ac;
          bc = h.ord_bc;
          if (p.trunc) {
            H.a_sa = h.ord_sa;
            H.b_tb = h.ord_tb;
          }
        }
        H.cap = p.nbuckets * p.bm + p.ovcap;   // compaction reads buckets and overflow
        H.max_probe = p.ovcap;
        if (e == hipSuccess) e = launch_zero(h.table, (size_t)16 * H.cap, stream);
        if (e == hipSuccess)
          e = launch_hash_laurent_bucket(H, G, dtype, ak, ac, na, bk, bc, nb,
                                         ctx->tune.hash_rows, stream);
      } else {
        if (e == hipSuccess)
          e = launch_zero(h.table, (size_t)(p.cw == 2 ? 32 : 16) * p.cap, stream);
        if (e == hipSuccess)
          e = launch_hash_laurent(H, dtype, a_codes, a_coef, na, b_codes, b_coef, nb,
                                  ctx->tune.hash_rows, stream);
      }
      if (e == hipSuccess) e = launch_hash_compact(H, dtype, stream);
    }
    if (e == hipSuccess) e = launch_finalize(h.meta, out_cap, out_n, &ctx->status->err, stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_mul_laurent launch");
  return KP_OK;
}

// Decoded output of a Poisson product: the grouped-products hash path writes
// it directly (and sets `decoded`), the others write keys.
struct PoissonOut {
  int32_t* x;
  int32_t* y;
  uint8_t* sin;
  DevLayout dec;
  bool decoded;
};

kp_status enqueue_poisson(kp_ctx* ctx, const kp_layout* layout, kp_mode mode,
                          const int64_t* a_x, const int64_t* a_y, const uint8_t* a_sin,
                          const double* a_coef, int64_t na, const int64_t* b_x,
                          const int64_t* b_y, const uint8_t* b_sin, const double* b_coef,
                          int64_t nb, int64_t* out_keys, double* out_coef, int64_t out_cap,
                          int64_t* out_n, void* workspace, size_t workspace_bytes,
                          hipStream_t stream, bool timed, PoissonOut* po = nullptr) {
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (layout && layout->ny == 0) return fail(ctx, KP_E_ARG, "kp_mul_poisson: layout has ny == 0");
  if (ctx->trunc_on)
    return fail(ctx, KP_E_ARG, "truncation by degree applies to Laurent products only");
  Plan p;
  kp_status st = make_plan(ctx, layout, 1, KP_F64, mode, na, nb, &p);
  if (st != KP_OK) return st;
  if (!out_n || out_cap < 0 || (na > 0 && (!a_x || !a_y || !a_sin || !a_coef)) ||
      (nb > 0 && (!b_x || !b_y || !b_sin || !b_coef)) || (out_cap > 0 && (!out_keys || !out_coef)))
    return fail(ctx, KP_E_ARG, "kp_mul_poisson: null array or negative capacity");
  if (workspace_bytes < p.ws || (p.ws > 0 && !workspace))
    return fail(ctx, KP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, p.ws);
  Carver c;
  c.base = static_cast<char*>(workspace);
  if (p.mode == KP_DENSE) {
    DenseBufs B{};
    carve_dense<true>(c, p, na, 2 * nb, &B);
    PoissonDenseBufs q{};
    carve_poisson_dense<true>(c, na, nb, &q);
    const PoissonDense pq = poisson_dense_codes(layout);
    B.a_keys_in = q.a_codes;
    B.a_coef_in = reinterpret_cast<const int64_t*>(q.a_coef);
    B.b_keys_in = q.b_codes;
    B.b_coef_in = reinterpret_cast<const int64_t*>(q.b_coef);
    B.ctx_err = &ctx->status->err;
    hipError_t e = launch_meta_init(B.meta, stream);
    if (na > 0 && nb > 0 && layout->nkeys > 0) {
      if (timed) std::tie(B.ev0, B.ev1) = timing_pair(ctx);
      if (e == hipSuccess)
        e = launch_poisson_dense_prep(layout->Wx, pq.N, pq.Hya, pq.Hyb, a_x, a_y, a_sin, a_coef,
                                      na, b_x, b_y, b_sin, b_coef, nb, q.a_codes, q.a_coef,
                                      q.b_codes, q.b_coef, stream);
      if (e == hipSuccess) e = launch_zero(B.dense, (size_t)8 * p.dp.nwin * p.dp.S, stream);
      if (e == hipSuccess) e = launch_dense_laurent(p.dp, B, KP_F64, stream);
      if (e == hipSuccess)
        e = launch_poisson_fold(layout->Wx, layout->Hy, pq.N, reinterpret_cast<const double*>(B.dense),
                                B.meta, out_keys, out_coef, out_cap, stream);
    }
    if (e == hipSuccess) e = launch_finalize(B.meta, out_cap, out_n, &ctx->status->err, stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "kp_mul_poisson launch");
    return KP_OK;
  }
  HashCarve h;
  carve_hash(c, p, 1, na, nb, &h);
  HashBufs H{h.meta, h.table, p.cap, p.cap, out_keys, out_coef, out_cap,
             nullptr, nullptr, hash_stats_ptr(ctx)};
  hipError_t e = launch_meta_init(h.meta, stream);
  if (na > 0 && nb > 0 && layout->nkeys > 0 && p.radix) {
    if (timed) std::tie(H.ev0, H.ev1) = timing_pair(ctx);
    const DevLayout dec = make_dev_layout(*layout, 0);
    if (e == hipSuccess)
      e = launch_poisson_prep(layout->Wx, a_x, a_y, a_sin, na, b_x, b_y, b_sin, nb, h.pp, stream,
                              p.harm ? &dec : nullptr, p.harm ? &ctx->harm : nullptr);
    RadixArgs R{nullptr, a_coef, na, nullptr, b_coef, nb, layout->Wx, h.pp, p.rows, p.l1,
                p.l2, 0, h.counts, h.pstart, h.bstart, h.ent1, h.ent2, h.meta, out_keys,
                out_coef, out_cap, H.stats, H.ev0, H.ev1};
    R.bin_log = p.blog;
    R.bin1 = h.bin1;
    R.dec = dec;
    if (p.harm) {
      R.harm_on = 1;
      R.harm = ctx->harm;
      R.harm_exact = p.harm_exact ? 1 : 0;
    }
    if (po) {
      R.out_x = po->x;
      R.out_y = po->y;
      R.out_t = po->sin;
      R.dec = po->dec;
      po->decoded = true;
    }
    if (e == hipSuccess) e = launch_radix(R, 2, stream);
  } else if (na > 0 && nb > 0 && layout->nkeys > 0) {
    if (timed) std::tie(H.ev0, H.ev1) = timing_pair(ctx);
    if (e == hipSuccess) e = launch_zero(h.table, (size_t)16 * p.cap, stream);
    if (e == hipSuccess)
      e = launch_poisson_prep(layout->Wx, a_x, a_y, a_sin, na, b_x, b_y, b_sin, nb, h.pp, stream);
    if (e == hipSuccess)
      e = launch_hash_poisson(H, layout->Wx, h.pp, a_coef, na, b_coef, nb, ctx->tune.hash_rows,
                              stream);
    if (e == hipSuccess) e = launch_hash_compact(H, KP_F64, stream);
  }
  if (e == hipSuccess) e = launch_finalize(h.meta, out_cap, out_n, &ctx->status->err, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_mul_poisson launch");
  return KP_OK;
}

kp_status enqueue_desc(kp_ctx* ctx, const kp_mul_desc& d, hipStream_t stream) {
  if (d.kind == KP_KIND_POISSON)
    return enqueue_poisson(ctx, &d.layout, d.mode, d.a_codes, d.a_y, d.a_sin,
                           (const double*)d.a_coef, d.na, d.b_codes, d.b_y, d.b_sin,
                           (const double*)d.b_coef, d.nb, d.out_codes, (double*)d.out_coef,
                           d.out_cap, d.out_n, d.workspace, d.workspace_bytes, stream, false);
  return enqueue_laurent(ctx, &d.layout, d.dtype, d.mode, d.a_codes, d.a_coef, d.na, d.b_codes,
                         d.b_coef, d.nb, d.out_codes, d.out_coef, d.out_cap, d.out_n, d.workspace,
                         d.workspace_bytes, stream, false);
}

}  // namespace
}  // namespace kp

kp_status kp_mul_laurent(kp_ctx* ctx, const kp_layout* layout, kp_dtype dtype, kp_mode mode,
                         unsigned flags, const int64_t* a_codes, const void* a_coef, int64_t na,
                         const int64_t* b_codes, const void* b_coef, int64_t nb,
                         int64_t* out_codes, void* out_coef, int64_t out_cap, int64_t* out_n,
                         void* workspace, size_t workspace_bytes, hipStream_t stream) {
  kp_status st = kp::enqueue_laurent(ctx, layout, dtype, mode, a_codes, a_coef, na, b_codes,
                                     b_coef, nb, out_codes, out_coef, out_cap, out_n, workspace,
                                     workspace_bytes, stream, true);
  if (st != KP_OK) return st;
  return kp::finish(ctx, flags, stream, "kp_mul_laurent");
}

kp_status kp_mul_laurent_noalloc(kp_ctx* ctx, const kp_layout* layout, kp_dtype dtype,
                                 kp_mode mode, unsigned flags, const int64_t* a_codes,
                                 const void* a_coef, int64_t na, const int64_t* b_codes,
                                 const void* b_coef, int64_t nb, int64_t* out_codes,
                                 void* out_coef, int64_t out_cap, int64_t* out_n,
                                 hipStream_t stream) {
  using namespace kp;
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (!ctx->scratch)
    return fail(ctx, KP_E_DEVICE, "kp_mul_laurent_noalloc: no scratch array on device %d (%s)",
                ctx->device, hipGetErrorString(ctx->scratch_err));
  Plan p;
  kp_status st = make_plan(ctx, layout, 0, dtype, mode, na, nb, &p);
  if (st != KP_OK) return st;
  if (p.ws > KP_SCRATCH_BYTES)
    return fail(ctx, KP_E_WORKSPACE,
                "kp_mul_laurent_noalloc: the product needs %zu bytes of workspace, the scratch "
                "array holds %zu",
                p.ws, (size_t)KP_SCRATCH_BYTES);
  // no timing events (creating them may allocate); the kernels see the
  // scratch array only through its device address
  st = kp::enqueue_laurent(ctx, layout, dtype, mode, a_codes, a_coef, na, b_codes, b_coef, nb,
                           out_codes, out_coef, out_cap, out_n, ctx->scratch, KP_SCRATCH_BYTES,
                           stream, false);
  if (st != KP_OK) return st;
  return kp::finish(ctx, flags, stream, "kp_mul_laurent_noalloc");
}

kp_status kp_mul_poisson(kp_ctx* ctx, const kp_layout* layout, kp_mode mode, unsigned flags,
                         const int64_t* a_x, const int64_t* a_y, const uint8_t* a_sin,
                         const double* a_coef, int64_t na, const int64_t* b_x,
                         const int64_t* b_y, const uint8_t* b_sin, const double* b_coef,
                         int64_t nb, int64_t* out_keys, double* out_coef, int64_t out_cap,
                         int64_t* out_n, void* workspace, size_t workspace_bytes,
                         hipStream_t stream) {
  kp_status st = kp::enqueue_poisson(ctx, layout, mode, a_x, a_y, a_sin, a_coef, na, b_x, b_y,
                                     b_sin, b_coef, nb, out_keys, out_coef, out_cap, out_n,
                                     workspace, workspace_bytes, stream, true);
  if (st != KP_OK) return st;
  return kp::finish(ctx, flags, stream, "kp_mul_poisson");
}

// ------------------------------------------------------------ from exponents
kp_status kp_plan_laurent(kp_ctx* ctx, int32_t nvars, kp_dtype dtype, kp_mode mode,
                          const int32_t* a_exps, int64_t na, const int32_t* b_exps, int64_t nb,
                          kp_layout* layout, kp_mode* resolved, int64_t* max_out_terms,
                          size_t* workspace_bytes, hipStream_t stream) {
  using namespace kp;
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (nvars < 1 || nvars > KP_MAX_VARS || na < 0 || nb < 0 || (na > 0 && !a_exps) ||
      (nb > 0 && !b_exps) || !layout || !resolved || !max_out_terms || !workspace_bytes)
    return fail(ctx, KP_E_ARG, "kp_plan_laurent: bad arguments");
  const int32_t* vals[2] = {a_exps, b_exps};
  const int64_t n[2] = {na, nb};
  const int32_t nv[2] = {nvars, nvars};
  int32_t r[2 * BOX_SET];
  kp_status st = read_boxes(ctx, 2, vals, n, nv, r, stream);
  if (st != KP_OK) return st;
  st = kp_layout_product(nvars, 0, r, r + KP_MAX_VARS, r + BOX_SET, r + BOX_SET + KP_MAX_VARS,
                         nullptr, nullptr, layout);
  if (st != KP_OK) return fail(ctx, st, "kp_plan_laurent: the product's codes overflow");
  Plan p;
  st = make_plan(ctx, layout, 0, dtype, mode, na, nb, &p);
  if (st != KP_OK) return st;
  *resolved = p.mode;
  *max_out_terms = p.max_out;
  *workspace_bytes = exps_workspace(0, na, nb, p.max_out, p.ws);
  return KP_OK;
}

kp_status kp_mul_laurent_exps(kp_ctx* ctx, const kp_layout* layout, kp_dtype dtype, kp_mode mode,
                              unsigned flags, const int32_t* a_exps, const void* a_coef, int64_t na,
                              const int32_t* b_exps, const void* b_coef, int64_t nb,
                              int32_t* out_exps, void* out_coef, int64_t out_cap, int64_t* out_n,
                              int64_t* n_host, void* workspace, size_t workspace_bytes,
                              hipStream_t stream) {
  using namespace kp;
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (!layout || layout->ny != 0 || layout->nx < 1)
    return fail(ctx, KP_E_ARG, "kp_mul_laurent_exps: needs a Laurent layout");
  if (na < 0 || nb < 0 || out_cap < 0 || !out_n || (na > 0 && (!a_exps || !a_coef)) ||
      (nb > 0 && (!b_exps || !b_coef)) || (out_cap > 0 && (!out_exps || !out_coef)))
    return fail(ctx, KP_E_ARG, "kp_mul_laurent_exps: null array or negative size");
  Plan p;
  kp_status st = make_plan(ctx, layout, 0, dtype, mode, na, nb, &p);
  if (st != KP_OK) return st;
  const size_t need = exps_workspace(0, na, nb, p.max_out, p.ws);
  if (workspace_bytes < need || !workspace)
    return fail(ctx, KP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
  Carver c;
  c.base = static_cast<char*>(workspace);
  int64_t* ka = c.take<int64_t>(na);
  int64_t* kb = c.take<int64_t>(nb);
  const int64_t ncodes = std::min<int64_t>(out_cap, std::max<int64_t>(p.max_out, 1));
  int64_t* oc = c.take<int64_t>(std::max<int64_t>(p.max_out, 1));
  hipError_t e = hipSuccess;
  if (layout->nkeys > 0)   // an empty product encodes nothing
    e = launch_encode2(make_dev_layout(*layout, 0), make_dev_layout(*layout, 1), na, nb, a_exps,
                       nullptr, nullptr, ka, nullptr, b_exps, nullptr, nullptr, kb, nullptr,
                       &ctx->status->err, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_mul_laurent_exps encode");
  // dense mode decodes in its output copy and posts the count from its
  // output scan, so the host wakes before the copy has run
  const bool sync = !(flags & KP_FLAG_ASYNC);
  ExpsOut xo{out_exps, make_dev_layout(*layout, 0), ctx->mb_dev, sync ? next_seq(ctx) : 0, false,
             false};
  st = enqueue_laurent(ctx, layout, dtype, mode, ka, a_coef, na, kb, b_coef, nb, oc, out_coef,
                       ncodes, out_n, static_cast<char*>(workspace) + c.off,
                       workspace_bytes - c.off, stream, true, &xo);
  if (st != KP_OK) return st;
  if (!xo.decoded) {
    e = launch_decode_n(make_dev_layout(*layout, 0), 0, out_n, ncodes, oc, out_exps, nullptr,
                        nullptr, &ctx->status->err, stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "kp_mul_laurent_exps decode");
  }
  if (!sync) return finish(ctx, flags, stream, "kp_mul_laurent_exps");
  return wait_count(ctx, out_n, n_host, stream, "kp_mul_laurent_exps", xo.posted ? xo.seq : 0);
}

kp_status kp_mul_laurent_auto(kp_ctx* ctx, int32_t nvars, kp_dtype dtype, kp_mode mode,
                              unsigned flags, const int32_t* a_exps, const void* a_coef, int64_t na,
                              const int32_t* b_exps, const void* b_coef, int64_t nb,
                              int32_t* out_exps, void* out_coef, int64_t out_cap, int64_t* out_n,
                              int64_t* n_host, void* workspace, size_t workspace_bytes,
                              kp_layout* layout, int64_t* need_cap, size_t* need_workspace,
                              hipStream_t stream) {
  if (!need_cap || !need_workspace) return kp::fail(ctx, KP_E_ARG, "kp_mul_laurent_auto: null size");
  kp_mode resolved;
  int64_t max_out = 0;
  size_t ws = 0;
  kp_status st = kp_plan_laurent(ctx, nvars, dtype, mode, a_exps, na, b_exps, nb, layout,
                                 &resolved, &max_out, &ws, stream);
  if (st != KP_OK) return st;
  *need_cap = std::max<int64_t>(max_out, 1);
  *need_workspace = ws;
  if (out_cap < *need_cap || workspace_bytes < ws || !workspace) return KP_E_WORKSPACE;
  return kp_mul_laurent_exps(ctx, layout, dtype, mode, flags, a_exps, a_coef, na, b_exps, b_coef,
                             nb, out_exps, out_coef, out_cap, out_n, n_host, workspace,
                             workspace_bytes, stream);
}

kp_status kp_plan_poisson(kp_ctx* ctx, int32_t nx, int32_t ny, kp_mode mode, const int32_t* a_x,
                          const int32_t* a_y, int64_t na, const int32_t* b_x, const int32_t* b_y,
                          int64_t nb, kp_layout* layout, kp_mode* resolved,
                          int64_t* max_out_terms, size_t* workspace_bytes, hipStream_t stream) {
  using namespace kp;
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (nx < 0 || nx > KP_MAX_VARS || ny < 1 || ny > KP_MAX_VARS || na < 0 || nb < 0 ||
      (na > 0 && ((nx > 0 && !a_x) || !a_y)) || (nb > 0 && ((nx > 0 && !b_x) || !b_y)) ||
      !layout || !resolved || !max_out_terms || !workspace_bytes)
    return fail(ctx, KP_E_ARG, "kp_plan_poisson: bad arguments");
  const int32_t* vals[4] = {a_y, b_y, a_x, b_x};
  const int64_t n[4] = {na, nb, na, nb};
  const int32_t nv[4] = {ny, ny, nx, nx};
  int32_t r[4 * BOX_SET];
  kp_status st = read_boxes(ctx, nx > 0 ? 4 : 2, vals, n, nv, r, stream);
  if (st != KP_OK) return st;
  // trigonometric half-widths: the largest |multiplier| per variable
  int32_t ha[KP_MAX_VARS], hb[KP_MAX_VARS];
  for (int v = 0; v < ny; ++v) {
    const int64_t a = std::max<int64_t>({-(int64_t)r[v], r[KP_MAX_VARS + v], 0});
    const int64_t b = std::max<int64_t>({-(int64_t)r[BOX_SET + v], r[BOX_SET + KP_MAX_VARS + v], 0});
    if (a > INT32_MAX || b > INT32_MAX)
      return fail(ctx, KP_E_CODE_OVERFLOW, "kp_plan_poisson: multiplier out of range");
    ha[v] = (int32_t)a;
    hb[v] = (int32_t)b;
  }
  const int32_t* xa = r + 2 * BOX_SET;
  const int32_t* xb = r + 3 * BOX_SET;
  st = kp_layout_product(nx, ny, xa, xa + KP_MAX_VARS, xb, xb + KP_MAX_VARS, ha, hb, layout);
  if (st != KP_OK) return fail(ctx, st, "kp_plan_poisson: the product's keys overflow");
  if (na == 0 || nb == 0) layout->nkeys = 0;
  Plan p;
  st = make_plan(ctx, layout, 1, KP_F64, mode, na, nb, &p);
  if (st != KP_OK) return st;
  *resolved = p.mode;
  *max_out_terms = p.max_out;
  *workspace_bytes = exps_workspace(1, na, nb, p.max_out, p.ws);
  return KP_OK;
}

kp_status kp_mul_poisson_exps(kp_ctx* ctx, const kp_layout* layout, kp_mode mode, unsigned flags,
                              const int32_t* a_x, const int32_t* a_y, const uint8_t* a_sin,
                              const double* a_coef, int64_t na, const int32_t* b_x,
                              const int32_t* b_y, const uint8_t* b_sin, const double* b_coef,
                              int64_t nb, int32_t* out_x, int32_t* out_y, uint8_t* out_sin,
                              double* out_coef, int64_t out_cap, int64_t* out_n, int64_t* n_host,
                              void* workspace, size_t workspace_bytes, hipStream_t stream) {
  using namespace kp;
  if (!ctx) return KP_E_ARG;
  if (!ctx->status) return fail(ctx, KP_E_ARG, "host-only context");
  if (!layout || layout->ny < 1)
    return fail(ctx, KP_E_ARG, "kp_mul_poisson_exps: needs a layout with a trigonometric part");
  const bool hx = layout->nx > 0;
  if (na < 0 || nb < 0 || out_cap < 0 || !out_n ||
      (na > 0 && ((hx && !a_x) || !a_y || !a_sin || !a_coef)) ||
      (nb > 0 && ((hx && !b_x) || !b_y || !b_sin || !b_coef)) ||
      (out_cap > 0 && ((hx && !out_x) || !out_y || !out_sin || !out_coef)))
    return fail(ctx, KP_E_ARG, "kp_mul_poisson_exps: null array or negative size");
  Plan p;
  kp_status st = make_plan(ctx, layout, 1, KP_F64, mode, na, nb, &p);
  if (st != KP_OK) return st;
  const size_t need = exps_workspace(1, na, nb, p.max_out, p.ws);
  if (workspace_bytes < need || !workspace)
    return fail(ctx, KP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
  Carver c;
  c.base = static_cast<char*>(workspace);
  int64_t* kxa = c.take<int64_t>(na);
  int64_t* kya = c.take<int64_t>(na);
  int64_t* kxb = c.take<int64_t>(nb);
  int64_t* kyb = c.take<int64_t>(nb);
  const int64_t ncodes = std::min<int64_t>(out_cap, std::max<int64_t>(p.max_out, 1));
  int64_t* ok = c.take<int64_t>(std::max<int64_t>(p.max_out, 1));
  hipError_t e = hipSuccess;
  if (layout->nkeys > 0)
    e = launch_encode2(make_dev_layout(*layout, 0), make_dev_layout(*layout, 1), na, nb, a_x, a_y,
                       a_sin, kxa, kya, b_x, b_y, b_sin, kxb, kyb, &ctx->status->err, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_mul_poisson_exps encode");
  PoissonOut po{out_x, out_y, out_sin, make_dev_layout(*layout, 0), false};
  st = enqueue_poisson(ctx, layout, mode, kxa, kya, a_sin, a_coef, na, kxb, kyb, b_sin, b_coef,
                       nb, ok, out_coef, ncodes, out_n, static_cast<char*>(workspace) + c.off,
                       workspace_bytes - c.off, stream, true, &po);
  if (st != KP_OK) return st;
  if (!po.decoded) {
    e = launch_decode_n(make_dev_layout(*layout, 0), 1, out_n, ncodes, ok, out_x, out_y, out_sin,
                        &ctx->status->err, stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "kp_mul_poisson_exps decode");
  }
  if (flags & KP_FLAG_ASYNC) return finish(ctx, flags, stream, "kp_mul_poisson_exps");
  return wait_count(ctx, out_n, n_host, stream, "kp_mul_poisson_exps");
}

// ------------------------------------------------------------ batches
struct kp_batch {
  kp_ctx* ctx = nullptr;
  int64_t max_tasks = 0;
  std::vector<kp_mul_desc> tasks;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last = nullptr;
};

namespace {
void drop_graph(kp_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}
}  // namespace

kp_status kp_batch_create(kp_ctx* ctx, int64_t max_tasks, kp_batch** out) {
  if (!ctx || !out || max_tasks < 1) return KP_E_ARG;
  if (!ctx->status) return kp::fail(ctx, KP_E_ARG, "host-only context");
  kp_batch* b = new (std::nothrow) kp_batch;
  if (!b) return kp::fail(ctx, KP_E_DEVICE, "out of host memory");
  b->ctx = ctx;
  b->max_tasks = max_tasks;
  b->tasks.reserve((size_t)max_tasks);
  *out = b;
  return KP_OK;
}

kp_status kp_batch_destroy(kp_batch* b) {
  if (!b) return KP_E_ARG;
  drop_graph(b);
  delete b;
  return KP_OK;
}

kp_status kp_batch_clear(kp_batch* b) {
  if (!b) return KP_E_ARG;
  drop_graph(b);
  b->tasks.clear();
  return KP_OK;
}

kp_status kp_batch_add(kp_batch* b, const kp_mul_desc* d, int64_t* task_id) {
  if (!b || !d) return KP_E_ARG;
  kp_ctx* ctx = b->ctx;
  if ((int64_t)b->tasks.size() >= b->max_tasks)
    return kp::fail(ctx, KP_E_ARG, "batch holds %lld tasks already", (long long)b->max_tasks);
  if (d->kind != KP_KIND_LAURENT && d->kind != KP_KIND_POISSON)
    return kp::fail(ctx, KP_E_ARG, "bad task kind %d", (int)d->kind);
  // host checks now, so that a launch queues only valid work
  kp::Plan p;
  kp_status st = kp::make_plan(ctx, &d->layout, d->kind == KP_KIND_POISSON,
                               d->kind == KP_KIND_POISSON ? KP_F64 : d->dtype, d->mode, d->na,
                               d->nb, &p);
  if (st != KP_OK) return st;
  if (!d->out_n || d->out_cap < 0 || (d->out_cap > 0 && (!d->out_codes || !d->out_coef)) ||
      (d->na > 0 && (!d->a_codes || !d->a_coef)) || (d->nb > 0 && (!d->b_codes || !d->b_coef)))
    return kp::fail(ctx, KP_E_ARG, "kp_batch_add: null array or negative capacity");
  if (d->kind == KP_KIND_POISSON && ((d->na > 0 && (!d->a_y || !d->a_sin)) ||
                                     (d->nb > 0 && (!d->b_y || !d->b_sin))))
    return kp::fail(ctx, KP_E_ARG, "kp_batch_add: null trigonometric array");
  if (d->workspace_bytes < p.ws || (p.ws > 0 && !d->workspace))
    return kp::fail(ctx, KP_E_WORKSPACE, "workspace of %zu bytes, %zu needed",
                    d->workspace_bytes, p.ws);
  drop_graph(b);
  b->tasks.push_back(*d);
  if (task_id) *task_id = (int64_t)b->tasks.size() - 1;
  return KP_OK;
}

kp_status kp_batch_launch(kp_batch* b, unsigned flags, hipStream_t stream) {
  if (!b) return KP_E_ARG;
  kp_ctx* ctx = b->ctx;
  hipError_t e = hipSuccess;
  if (flags & KP_BATCH_GRAPH) {
    if (!stream)
      return kp::fail(ctx, KP_E_ARG, "graph capture needs a stream other than the null stream");
    if (!b->exec) {
      // capture the queued work once; later launches replay it
      e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
      if (e != hipSuccess) return kp::hip_fail(ctx, e, "hipStreamBeginCapture");
      kp_status st = KP_OK;
      for (const kp_mul_desc& d : b->tasks) {
        st = kp::enqueue_desc(ctx, d, stream);
        if (st != KP_OK) break;
      }
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(stream, &g);
      if (st != KP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return kp::hip_fail(ctx, e, "hipStreamEndCapture");
      b->graph = g;
      e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        drop_graph(b);
        return kp::hip_fail(ctx, e, "hipGraphInstantiate");
      }
    }
    e = hipGraphLaunch(b->exec, stream);
    if (e != hipSuccess) return kp::hip_fail(ctx, e, "hipGraphLaunch");
  } else {
    for (const kp_mul_desc& d : b->tasks) {
      kp_status st = kp::enqueue_desc(ctx, d, stream);
      if (st != KP_OK) return st;
    }
  }
  b->last = stream;
  return kp::finish(ctx, KP_FLAG_ASYNC, stream, "kp_batch_launch");
}

kp_status kp_batch_status(kp_batch* b, int64_t task_id, int64_t* n_out) {
  if (!b || !n_out) return KP_E_ARG;
  if (task_id < 0 || task_id >= (int64_t)b->tasks.size())
    return kp::fail(b->ctx, KP_E_ARG, "no task %lld", (long long)task_id);
  hipError_t e = hipStreamSynchronize(b->last);
  if (e == hipSuccess)
    e = hipMemcpy(n_out, b->tasks[(size_t)task_id].out_n, sizeof(int64_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return kp::hip_fail(b->ctx, e, "kp_batch_status");
  return *n_out < 0 ? (kp_status)(-*n_out) : KP_OK;
}

// ------------------------------------------------------------ packed batches
struct kp_pack {
  kp_ctx* ctx = nullptr;
  int max_tasks = 0;
  size_t table_bytes = 0;
  void* table_dev = nullptr;        // device task table
  char* table_host = nullptr;       // pinned staging of the same bytes
  uint64_t* post = nullptr;         // pinned, mapped: boxes (2 arrays a task), then counts
  uint64_t* post_dev = nullptr;
  // box kernel arguments (pinned, mapped): arrays, lengths, variables
  const int32_t** box_vals = nullptr;
  int64_t* box_n = nullptr;
  int32_t* box_nv = nullptr;
  const int32_t** box_vals_dev = nullptr;
  int64_t* box_n_dev = nullptr;
  int32_t* box_nv_dev = nullptr;
  uint64_t seq = 0;
  // the planned batch
  std::vector<kp_pack_task> tasks;
  std::vector<kp_layout> layouts;
  std::vector<int64_t> caps, slots, off;
  std::vector<int32_t> direct;
  size_t arena = 0;
  bool running = false;
  hipStream_t run_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {
constexpr int PACK_MAX = 4096;

size_t pack_post_words(int max_tasks) {
  return (size_t)max_tasks * 2 * 2 * KP_MAX_VARS + 2 * (size_t)max_tasks;
}

void pack_free(kp_pack* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->table_dev) (void)hipFree(p->table_dev);
  if (p->table_host) (void)hipHostFree(p->table_host);
  if (p->post) (void)hipHostFree(p->post);
  if (p->box_vals) (void)hipHostFree(p->box_vals);
  delete p;
}

// Waits until every word of post[0..n) carries `tag` in its high half.
kp_status pack_wait_words(kp_pack* p, const uint64_t* w, size_t n, uint64_t tag, hipStream_t s,
                          const char* what) {
  for (size_t i = 0; i < n; ++i) {
    kp_status st = kp::wait_tag(p->ctx, w + i, tag, s, what);
    if (st != KP_OK) return st;
  }
  return KP_OK;
}
}  // namespace

kp_status kp_pack_create(kp_ctx* ctx, int32_t max_tasks, kp_pack** out) {
  if (!ctx || !out) return KP_E_ARG;
  if (!ctx->status) return kp::fail(ctx, KP_E_ARG, "host-only context");
  if (max_tasks < 1 || max_tasks > PACK_MAX)
    return kp::fail(ctx, KP_E_ARG, "kp_pack_create: 1..%d tasks", PACK_MAX);
  kp_pack* p = new (std::nothrow) kp_pack;
  if (!p) return kp::fail(ctx, KP_E_DEVICE, "out of host memory");
  p->ctx = ctx;
  p->max_tasks = max_tasks;
  p->table_bytes = kp::pack_table_bytes(max_tasks);
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e == hipSuccess) e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc(&p->table_dev, p->table_bytes);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&p->table_host), p->table_bytes);
  const size_t pw = pack_post_words(max_tasks);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&p->post), pw * sizeof(uint64_t),
                      hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) {
    std::memset(p->post, 0, pw * sizeof(uint64_t));
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&p->post_dev), p->post, 0);
  }
  const size_t segs = 2 * (size_t)max_tasks;
  const size_t box_bytes = segs * (sizeof(void*) + sizeof(int64_t) + sizeof(int32_t));
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&p->box_vals), box_bytes,
                      hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) {
    p->box_n = reinterpret_cast<int64_t*>(p->box_vals + segs);
    p->box_nv = reinterpret_cast<int32_t*>(p->box_n + segs);
    char* dev = nullptr;
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&dev), p->box_vals, 0);
    if (e == hipSuccess) {
      p->box_vals_dev = reinterpret_cast<const int32_t**>(dev);
      p->box_n_dev = reinterpret_cast<int64_t*>(dev + segs * sizeof(void*));
      p->box_nv_dev = reinterpret_cast<int32_t*>(dev + segs * (sizeof(void*) + sizeof(int64_t)));
    }
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    pack_free(p);
    return kp::hip_fail(ctx, e, "kp_pack_create");
  }
  *out = p;
  return KP_OK;
}

kp_status kp_pack_destroy(kp_pack* p) {
  if (!p) return KP_E_ARG;
  if (p->running && p->run_stream) (void)hipStreamSynchronize(p->run_stream);
  pack_free(p);
  return KP_OK;
}

kp_status kp_pack_plan(kp_pack* p, const kp_pack_task* tasks, int32_t n, int64_t* out_cap,
                       size_t* arena_bytes, hipStream_t stream) {
  using namespace kp;
  if (!p) return KP_E_ARG;
  kp_ctx* ctx = p->ctx;
  if (p->running) return fail(ctx, KP_E_ARG, "kp_pack_plan: the last run was not waited for");
  if (n < 0 || n > p->max_tasks || (n > 0 && (!tasks || !out_cap)) || !arena_bytes)
    return fail(ctx, KP_E_ARG, "kp_pack_plan: bad arguments (at most %d tasks)", p->max_tasks);
  for (int32_t k = 0; k < n; ++k) {
    const kp_pack_task& t = tasks[k];
    if (t.nvars < 1 || t.nvars > KP_MAX_VARS || t.na < 0 || t.nb < 0 ||
        t.na >= ((int64_t)1 << 31) || t.nb >= ((int64_t)1 << 31) ||
        (t.na > 0 && (!t.a_exps || !t.a_coef)) || (t.nb > 0 && (!t.b_exps || !t.b_coef)))
      return fail(ctx, KP_E_ARG, "kp_pack_plan: task %d has bad sizes or null arrays", (int)k);
    if (t.dtype != KP_I64 && t.dtype != KP_F64)
      return fail(ctx, KP_E_DTYPE, "kp_pack_plan: task %d: int64 or fp64 coefficients", (int)k);
  }
  p->tasks.assign(tasks, tasks + n);
  p->layouts.assign((size_t)n, kp_layout{});
  p->caps.assign((size_t)n, 0);
  p->slots.assign((size_t)n, 0);
  p->direct.assign((size_t)n, 0);
  p->off.assign((size_t)n, 0);
  p->arena = 0;
  // every factor's box: one launch, one wait
  int nseg = 0;
  for (int32_t k = 0; k < n; ++k)
    for (int f = 0; f < 2; ++f) {
      const kp_pack_task& t = tasks[k];
      p->box_vals[nseg] = f ? t.b_exps : t.a_exps;
      p->box_n[nseg] = f ? t.nb : t.na;
      p->box_nv[nseg] = t.nvars;
      ++nseg;
    }
  if (++p->seq == 0 || (uint32_t)p->seq == 0) p->seq += 1;
  const uint64_t tag = (uint64_t)(uint32_t)p->seq;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipError_t e = launch_pack_boxes(p->box_vals_dev, p->box_n_dev, p->box_nv_dev, nseg,
                                   p->post_dev, p->seq, stream);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_pack_plan boxes");
  size_t arena = 0;
  for (int32_t k = 0; k < n; ++k) {
    const kp_pack_task& t = tasks[k];
    int32_t box[2][2 * KP_MAX_VARS];
    for (int f = 0; f < 2; ++f) {
      const int g = 2 * k + f;
      const uint64_t* w = p->post + (size_t)g * 2 * KP_MAX_VARS;
      const bool empty = (f ? t.nb : t.na) == 0;
      for (int v = 0; v < t.nvars; ++v)
        for (int side = 0; side < 2; ++side) {
          int32_t x = side ? -1 : 0;   // an empty array: min 0, max -1
          if (!empty) {
            const uint64_t* slot = w + side * KP_MAX_VARS + v;
            kp_status st = wait_tag(ctx, slot, tag, stream, "kp_pack_plan boxes");
            if (st != KP_OK) return st;
            x = (int32_t)(uint32_t)__atomic_load_n(slot, __ATOMIC_ACQUIRE);
          }
          box[f][side * KP_MAX_VARS + v] = x;
        }
    }
    kp_layout& L = p->layouts[(size_t)k];
    kp_status st = kp_layout_product(t.nvars, 0, box[0], box[0] + KP_MAX_VARS, box[1],
                                     box[1] + KP_MAX_VARS, nullptr, nullptr, &L);
    if (st != KP_OK)
      return fail(ctx, st, "kp_pack_plan: task %d: the product's codes overflow", (int)k);
    // bound on result terms; a hash table of at least twice as many slots, or
    // one word per code when that is no larger
    const int64_t pairs = t.na * t.nb;
    const int64_t bound = L.nkeys <= 0 ? 0 : std::min<int64_t>(L.nkeys, pairs);
    int64_t hs = 64;
    while (hs < 2 * bound) hs <<= 1;
    const bool dir = L.nkeys > 0 && L.nkeys <= 2 * hs;
    p->caps[(size_t)k] = bound;
    p->slots[(size_t)k] = bound == 0 ? 0 : (dir ? L.nkeys : hs);
    p->direct[(size_t)k] = dir ? 1 : 0;
    p->off[(size_t)k] = (int64_t)arena;
    const int64_t words = p->direct[(size_t)k] ? p->slots[(size_t)k] : 2 * p->slots[(size_t)k];
    arena += align_up(8 * (size_t)t.na) + align_up(8 * (size_t)t.nb) +
             align_up(8 * (size_t)std::max<int64_t>(words, 1)) + ALIGN;
    out_cap[k] = bound;
  }
  p->arena = arena;
  *arena_bytes = arena;
  return KP_OK;
}

kp_status kp_pack_run(kp_pack* p, int32_t* const* out_exps, void* const* out_coef, void* arena,
                      size_t arena_bytes, unsigned flags, hipStream_t stream) {
  using namespace kp;
  if (!p) return KP_E_ARG;
  kp_ctx* ctx = p->ctx;
  const int n = (int)p->tasks.size();
  if (p->running) return fail(ctx, KP_E_ARG, "kp_pack_run: the last run was not waited for");
  if (arena_bytes < p->arena || (p->arena > 0 && !arena) || (n > 0 && (!out_exps || !out_coef)))
    return fail(ctx, KP_E_WORKSPACE, "kp_pack_run: arena of %zu bytes, %zu needed", arena_bytes,
                p->arena);
  for (int k = 0; k < n; ++k)
    if (p->caps[(size_t)k] > 0 && (!out_exps[k] || !out_coef[k]))
      return fail(ctx, KP_E_ARG, "kp_pack_run: task %d has no output arrays", k);
  if ((flags & KP_PACK_GRAPH) && !stream)
    return fail(ctx, KP_E_ARG, "graph capture needs a stream other than the null stream");
  // the table: header, unit prefixes, tasks
  const int m = p->max_tasks;
  PackHeader* h = reinterpret_cast<PackHeader*>(p->table_host);
  int64_t* pre = reinterpret_cast<int64_t*>(p->table_host + sizeof(PackHeader));
  int64_t* pre_prep = pre;
  int64_t* pre_mul = pre + (m + 1);
  int64_t* pre_cmp = pre + 2 * (m + 1);
  PackTask* tt = reinterpret_cast<PackTask*>(pre + 3 * (m + 1));
  if (++p->seq == 0 || (uint32_t)p->seq == 0) p->seq += 1;
  h->ntasks = n;
  h->max_tasks = m;
  h->err = 0;
  h->pad = 0;
  h->seq = p->seq;
  h->post = p->post_dev + (size_t)m * 2 * 2 * KP_MAX_VARS;
  pre_prep[0] = pre_mul[0] = pre_cmp[0] = 0;
  char* base = static_cast<char*>(arena);
  for (int k = 0; k < n; ++k) {
    const kp_pack_task& t = p->tasks[(size_t)k];
    const size_t K = (size_t)k;
    PackTask& T = tt[k];
    T.la = make_dev_layout(p->layouts[K], 0);
    T.lb = make_dev_layout(p->layouts[K], 1);
    T.ax = t.a_exps;
    T.bx = t.b_exps;
    T.ac = t.a_coef;
    T.bc = t.b_coef;
    T.na = t.na;
    T.nb = t.nb;
    char* q = base + p->off[K];
    T.ak = reinterpret_cast<int64_t*>(q);
    q += align_up(8 * (size_t)t.na);
    T.bk = reinterpret_cast<int64_t*>(q);
    q += align_up(8 * (size_t)t.nb);
    T.table = reinterpret_cast<uint64_t*>(q);
    T.slots = p->slots[K];
    T.direct = p->direct[K];
    const int64_t words = T.direct ? T.slots : 2 * T.slots;
    q += align_up(8 * (size_t)std::max<int64_t>(words, 1));
    T.count = reinterpret_cast<unsigned long long*>(q);
    T.f64 = t.dtype == KP_F64 ? 1 : 0;
    T.out_x = p->caps[K] > 0 ? out_exps[k] : nullptr;
    T.out_c = p->caps[K] > 0 ? out_coef[k] : nullptr;
    T.out_cap = p->caps[K];
    // multiply units: rows of A by blocks of PACK_BLOCK terms of B, about
    // 2^14 pairs each
    const int64_t bw = std::min<int64_t>(std::max<int64_t>(t.nb, 1), PACK_BLOCK);
    T.rows = std::max<int64_t>(1, std::min<int64_t>(std::max<int64_t>(t.na, 1), 16384 / bw));
    T.bblocks = (t.nb + PACK_BLOCK - 1) / PACK_BLOCK;
    const int64_t live = p->caps[K] > 0 ? 1 : 0;   // an empty product makes no pairs
    const int64_t enc = (t.na + PACK_BLOCK - 1) / PACK_BLOCK + (t.nb + PACK_BLOCK - 1) / PACK_BLOCK;
    const int64_t clr = std::max<int64_t>(1, (words + 4 * PACK_BLOCK - 1) / (4 * PACK_BLOCK));
    const int64_t mul = live * ((t.na + T.rows - 1) / T.rows) * T.bblocks;
    const int64_t cmp = (T.slots + 8 * PACK_BLOCK - 1) / (8 * PACK_BLOCK);
    pre_prep[k + 1] = pre_prep[k] + live * enc + clr;
    pre_mul[k + 1] = pre_mul[k] + mul;
    pre_cmp[k + 1] = pre_cmp[k] + cmp;
    if (!live) {   // nothing to encode: the prep units are the clearing ones
      T.na = T.nb = 0;
    }
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  const int grid = std::max(1, ctx->num_cu * 4);
  hipError_t e = hipSuccess;
  if (flags & KP_PACK_GRAPH) {
    if (!p->exec) {
      // the upload and the four stages, captured once: the kernels read
      // everything from the table, so every later batch replays them
      e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
      if (e == hipSuccess) {
        hipError_t e1 = hipMemcpyAsync(p->table_dev, p->table_host, p->table_bytes,
                                       hipMemcpyHostToDevice, stream);
        if (e1 == hipSuccess) e1 = launch_pack_run(p->table_dev, grid, stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(stream, &g);
        if (e1 != hipSuccess) e = e1;
        if (e == hipSuccess) {
          p->graph = g;
          e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
        } else if (g) {
          (void)hipGraphDestroy(g);
        }
      }
    }
    if (e == hipSuccess) e = hipGraphLaunch(p->exec, stream);
  } else {
    e = hipMemcpyAsync(p->table_dev, p->table_host, p->table_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_pack_run(p->table_dev, grid, stream);
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return hip_fail(ctx, e, "kp_pack_run");
  p->running = true;
  p->run_stream = stream;
  return KP_OK;
}

kp_status kp_pack_wait(kp_pack* p, int64_t* n_out) {
  using namespace kp;
  if (!p) return KP_E_ARG;
  const int n = (int)p->tasks.size();
  if (!p->running) return fail(p->ctx, KP_E_ARG, "kp_pack_wait: nothing is running");
  if (n > 0 && !n_out) return fail(p->ctx, KP_E_ARG, "kp_pack_wait: null counts");
  const uint64_t tag = (uint64_t)(uint32_t)p->seq;
  const uint64_t* w = p->post + (size_t)p->max_tasks * 2 * 2 * KP_MAX_VARS;
  kp_status st = pack_wait_words(p, w, 2 * (size_t)n, tag, p->run_stream, "kp_pack_wait");
  p->running = false;
  if (st != KP_OK) return st;
  kp_status first = KP_OK;
  for (int k = 0; k < n; ++k) {
    const uint64_t lo = __atomic_load_n(w + 2 * k, __ATOMIC_ACQUIRE) & 0xffffffffu;
    const uint64_t hi = __atomic_load_n(w + 2 * k + 1, __ATOMIC_ACQUIRE) & 0xffffffffu;
    n_out[k] = (int64_t)((hi << 32) | lo);
    if (n_out[k] < 0 && first == KP_OK) first = (kp_status)(-n_out[k]);
  }
  if (first != KP_OK) return fail(p->ctx, first, "kp_pack_wait: a task reported a device error");
  return KP_OK;
}

kp_status kp_pack_query(kp_pack* p, int32_t* done) {
  if (!p || !done) return KP_E_ARG;
  if (!p->running) {
    *done = 1;
    return KP_OK;
  }
  const int n = (int)p->tasks.size();
  const uint64_t tag = (uint64_t)(uint32_t)p->seq;
  const uint64_t* w = p->post + (size_t)p->max_tasks * 2 * 2 * KP_MAX_VARS;
  *done = 1;
  for (int k = 0; k < 2 * n; ++k)
    if ((__atomic_load_n(w + k, __ATOMIC_ACQUIRE) >> 32) != tag) {
      *done = 0;
      break;
    }
  if (!*done) {
    // a stream that failed or finished without posting ends the wait
    const hipError_t q = hipStreamQuery(p->run_stream);
    if (q != hipSuccess && q != hipErrorNotReady) return kp::hip_fail(p->ctx, q, "kp_pack_query");
  }
  return KP_OK;
}

kp_status kp_encode_host(const kp_layout* layout, int which, int64_t n, const int32_t* x_exps,
                         const int32_t* y_mult, const uint8_t* is_sin, int64_t* xcodes,
                         int64_t* ycodes) {
  if (!layout || (which != 0 && which != 1) || n < 0) return KP_E_ARG;
  if (n > 0 && ((layout->nx > 0 && !x_exps) || !xcodes ||
                (layout->ny > 0 && (!y_mult || !is_sin || !ycodes))))
    return KP_E_ARG;
  DevLayout d = make_dev_layout(*layout, which);
  uint32_t err = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t kx = 0, ky = 0;
    err |= encode_term(d, x_exps + i * d.nx, d.ny ? y_mult + i * d.ny : nullptr,
                       d.ny ? is_sin[i] : 0, &kx, &ky);
    xcodes[i] = kx;
    if (d.ny) ycodes[i] = ky;
  }
  return (kp_status)first_error(err);
}

kp_status kp_decode_host(const kp_layout* layout, int poisson, int64_t n, const int64_t* codes,
                         int32_t* x_exps, int32_t* y_mult, uint8_t* is_sin) {
  if (!layout || n < 0) return KP_E_ARG;
  if (poisson && layout->ny == 0) return KP_E_ARG;
  if (n > 0 && (!codes || (layout->nx > 0 && !x_exps) || (poisson && (!y_mult || !is_sin))))
    return KP_E_ARG;
  DevLayout d = make_dev_layout(*layout, 0);
  uint32_t err = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = codes[i];
    if (c < 0 || c >= d.nkeys) {
      err |= ERR_RANGE;
      c = 0;
    }
    uint64_t q = (uint64_t)c;
    if (poisson) {
      is_sin[i] = (uint8_t)(q & 1);
      q >>= 1;
      uint64_t u = fdiv(q, d.dWx);
      decode_x(d, q - u * (uint64_t)d.Wx, x_exps + i * d.nx);
      decode_y(d, u, y_mult + i * d.ny);
    } else {
      decode_x(d, q, x_exps + i * d.nx);
    }
  }
  return (kp_status)first_error(err);
}

}  // extern "C"
