/*
 * kp.h -- C ABI of the MI355X (gfx950) Kronecker sparse-multiply library.
 *
 * Multiplies sparse multivariate Laurent polynomials and Poisson series the
 * way Biscani (ISSAC 2010) describes: generalised Kronecker substitution
 * turns every multi-index into one integer code (Section 2, Tables 1-2,
 * c(e) = c.e - chi), the schoolbook method forms every term-by-term product
 * (Section 3), and the products are accumulated by code either in a dense
 * code-indexed array (Section 3.1, "moderately sparse") or in a hash table
 * keyed by code (Section 3.2, "highly sparse").  Poisson series split each
 * trigonometric product into cos/sin of the sum and of the difference of the
 * arguments (Section 2, eq. werner, with the factor 1/2 the printed formulas
 * leave out).
 *
 * Conventions common to every entry point
 *  - All functions are extern "C", never throw, and return a kp_status.
 *  - Pointers documented as "device" point to HIP device memory owned by the
 *    caller (for example torch tensors); "host" pointers are ordinary memory.
 *    The library never allocates or frees caller-visible device memory: its
 *    own device memory is a 256-byte status block per context and the
 *    scratch array of kp_mul_laurent_noalloc (one per GPU, static).
 *  - Every launch is ordered on the given hipStream_t (0 = null stream).
 *  - Without KP_FLAG_ASYNC a call synchronises its stream once and reports
 *    device-detected errors (range, capacity) in its return value.  With it,
 *    the call returns after queuing; device errors are latched in the
 *    context's status block (read and cleared by kp_ctx_check) and, for
 *    multiplies, the device count *out_n is set to -(status) instead of the
 *    term count.  A multiply also reports, through *out_n, an error that an
 *    earlier asynchronous call on the same context latched and that has not
 *    been cleared (for example an exponent outside the box in kp_encode), so
 *    encode + multiply can be queued with one synchronisation at the end.
 *  - Host-detectable errors (bad arguments, layout overflow, workspace too
 *    small) return before anything is queued.
 *  - Exponent arrays are row-major int32 [n][nvars].
 */
#ifndef KP_H
#define KP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KP_MAX_VARS 16

typedef enum kp_status {
  KP_OK = 0,
  KP_E_ARG = 1,           /* invalid argument (null pointer, bad size, bad enum)      */
  KP_E_RANGE = 2,         /* an exponent or multiplier lies outside the layout's box   */
  KP_E_CODE_OVERFLOW = 3, /* the product box needs 2^62 codes or more (Section 2:
                             a code is unique only if the multi-index is representable) */
  KP_E_NONCANONICAL = 4,  /* Poisson input whose first nonzero multiplier is negative,
                             or a sine with the zero multiplier vector                  */
  KP_E_CAPACITY = 5,      /* out_cap smaller than the number of result terms, or a
                             forced hash capacity too small for the result              */
  KP_E_WORKSPACE = 6,     /* workspace smaller than kp_mul_bound asked for             */
  KP_E_DEVICE = 7,        /* the HIP runtime reported an error                         */
  KP_E_DTYPE = 8,         /* coefficient type not supported by this operation          */
  KP_E_MODE = 9           /* KP_DENSE requested for a box too large for dense mode     */
} kp_status;

/* Coefficient types.  KP_I64: int64 in and out, products and sums wrap
   modulo 2^64.  KP_F64: double in and out.  KP_I128 (Laurent only): int64
   coefficients in, every product formed exactly in 128 bits and summed in
   128-bit accumulators (Section 5: the 64-bit-input, 128-bit-output integer
   arithmetic the paper's Fateman timings compare against); each output
   coefficient is 16 bytes, the low then the high 64-bit word of the sum
   modulo 2^128: exact as a two's complement value while |sum| < 2^127, and
   as an unsigned value for nonnegative sums below 2^128 (the Fateman product
   at degree 30 has coefficients between 2^127 and 2^128).  Out-coefficient
   arrays hold out_cap * 16 bytes. */
typedef enum kp_dtype { KP_I64 = 0, KP_F64 = 1, KP_I128 = 2 } kp_dtype;

/* Accumulator choice (Section 3: dense array for moderately sparse products,
   hash table for highly sparse ones; the paper leaves the criterion to "an
   analysis of the densities").  KP_AUTO applies the context's rule. */
typedef enum kp_mode { KP_AUTO = 0, KP_DENSE = 1, KP_HASH = 2 } kp_mode;

enum { KP_FLAG_ASYNC = 1 };

/*
 * kp_layout: the coding vectors of one product (Section 2, Table 2).
 *
 * Polynomial (Laurent) variables x_0..x_{nx-1}: each factor term's exponent
 * e_k must lie in its factor's box [amin_k, amax_k] (factor A) or
 * [bmin_k, bmax_k] (factor B).  The product box is [amin_k+bmin_k,
 * amax_k+bmax_k] with width xw_k; x_0 is the least significant digit:
 * xc_0 = 1, xc_k = xc_{k-1} * xw_{k-1}, Wx = prod xw_k.  A factor term is
 * coded relative to its own factor's minimum, kx = sum_k xc_k (e_k - min_k),
 * so the code of a product term is simply kx_a + kx_b (that is, c.e - chi
 * with chi = c . e_min of the product box).
 *
 * Trigonometric multipliers y_0..y_{ny-1} (Poisson series only): factor
 * half-widths ha_k = max |ja_k|, hb_k = max |jb_k|; the product's balanced
 * box has yh_k = ha_k + hb_k and width 2*yh_k + 1, with y_0 the MOST
 * significant digit (yc_{ny-1} = 1).  ky = sum_k yc_k j_k is signed; adding
 * and subtracting codes adds and subtracts multiplier vectors (the extension
 * of the coding vector Section 2 calls for), and sign(ky) is the sign of the
 * first nonzero multiplier, so the canonical form is |ky| with a sign flip
 * of sines.  Hy = (prod(2 yh_k + 1) - 1) / 2 is the largest |ky|.
 *
 * nkeys: size of the product's key space.  Laurent: Wx.  Poisson:
 * 2 * Wx * (Hy + 1), a key being 2 * (kx + Wx * |ky|) + is_sin.
 */
typedef struct kp_layout {
  int32_t nx, ny;
  int32_t amin[KP_MAX_VARS], amax[KP_MAX_VARS];
  int32_t bmin[KP_MAX_VARS], bmax[KP_MAX_VARS];
  int32_t ha[KP_MAX_VARS], hb[KP_MAX_VARS];
  int64_t xmin[KP_MAX_VARS]; /* product box minimum amin_k + bmin_k             */
  int64_t xw[KP_MAX_VARS];   /* product widths                                  */
  int64_t xc[KP_MAX_VARS];   /* strides, x_0 least significant                  */
  int64_t Wx;                /* prod xw_k                                       */
  int64_t yh[KP_MAX_VARS];   /* balanced half-widths ha_k + hb_k                */
  int64_t yc[KP_MAX_VARS];   /* strides, y_0 most significant                   */
  int64_t Hy;                /* largest |ky|                                    */
  int64_t nkeys;             /* key-space size, < 2^62                          */
} kp_layout;

/* Tuning knobs (the paper leaves block size, table size and the density
   criterion unspecified).  None of them changes a result. */
typedef struct kp_tune {
  int32_t window;           /* dense: output codes per LDS window, a multiple of 2048
                               up to 18432 (default 18432)                           */
  int32_t block;            /* dense: threads per workgroup (256, 512 or 1024)       */
  int32_t tasks_per_cu;     /* dense: equal-cost tasks per compute unit (default 1)  */
  double hash_load;         /* hash: target load factor (0.05 .. 0.9)                */
  int64_t hash_capacity;    /* hash: forced slot count (0 = from the bound)          */
  int64_t dense_max_keys;   /* dense only if nkeys <= this (at most 2^27)            */
  double dense_keys_per_pair; /* auto mode: dense only if nkeys <= this * na * nb
                                 (default 8)                                          */
  int32_t hash_rows;        /* hash: factor-A rows per thread (global table)         */
  int32_t hash_partitioned; /* hash: 2 = products grouped by hash bits in two levels
                               through HBM, each group accumulated in an LDS table
                               (workspace 34 bytes per product); 0 = one open-addressing
                               table in HBM; 1 (default) = grouped when the products are
                               at most 4 times the result bound, else the table          */
  int32_t hash_bucket;      /* hash, Laurent, int64/fp64: > 0 selects Section 3.2's bucketed
                               table instead of the above, with this many slots per bucket
                               (1 .. 16): product code e goes to bucket e mod N, where it is
                               added to the slot holding e or appended; a full bucket sends
                               it to an overflow table (open addressing, six times the
                               codes expected to overflow if the bound's codes spread over
                               the buckets as a Poisson variable, at least 1024 slots); a
                               full overflow table is KP_E_CAPACITY.  0 (default) = not
                               used                                                       */
  int32_t hash_order;       /* bucketed table: 1 (default) orders both factors' terms by
                               code mod N first (Section 3.2's term order), 0 keeps them  */
  int32_t hash_bin_slots;   /* grouped products: slots of one bin's LDS table, 2048, 4096
                               (default) or 8192, 16 bytes each; bins are sized for half
                               a table of products on average.  KP_I128 sums use 24-byte
                               slots and at most 4096 of them (8192 acts as 4096); their
                               grouped entries carry the pair's 32-bit term indices, so
                               factors of 2^32 terms or more keep the global table        */
  int32_t hash_grouping;    /* grouped products, Laurent int64/fp64: 2 = grouped by output
                               code range (level 1 found from the sorted factors, so each
                               product is written once, to a hash bin of its range);
                               1 = two levels of hash bits through HBM (always used for
                               Poisson series and 128-bit sums); 0 (default) = by range
                               for products spread thinly over the code space (at most one
                               per 64 codes), else, and under a truncation (the two-level
                               grouping drops pairs over the limit before forming them),
                               two levels.  Either
                               way a bin whose distinct codes overflow its table is redone
                               in parts                                                   */
  int32_t hash_max_bin_bits; /* grouped by code range: at most 2^this bins per range (0..10,
                               default 10); fewer bins than the products ask for leave bins
                               that overflow their table and are redone in parts          */
  int32_t hash_bin_fill;    /* grouped by code range: products planned per bin, in percent
                               of the bin's table slots (10..90, default 42)              */
} kp_tune;

typedef struct kp_ctx kp_ctx;

/* Context: device id, tuning, last error text, a 256-byte device status
   block.  One context per host thread; not thread-safe.  device < 0 makes a
   host-only context (no device touched) that serves kp_mul_bound and the
   tuning calls; the launching entry points reject it with KP_E_ARG. */
kp_status kp_ctx_create(int device, kp_ctx** out);
kp_status kp_ctx_destroy(kp_ctx* ctx);
kp_status kp_ctx_get_tune(const kp_ctx* ctx, kp_tune* out);
kp_status kp_ctx_set_tune(kp_ctx* ctx, const kp_tune* tune);
/* Synchronise `stream`, return and clear the latched device status. */
kp_status kp_ctx_check(kp_ctx* ctx, hipStream_t stream);
const char* kp_status_str(kp_status s);
const char* kp_last_error(const kp_ctx* ctx);

/* Instrumentation.  While enabled, every multiply records a pair of HIP
   events on its stream around its accumulation kernel (the dense window
   kernel or the hash insert kernel).  kp_ctx_timing_read waits for those
   events, returns the summed kernel time in milliseconds and the number of
   timed launches, and clears the record.  Disabled by default. */
kp_status kp_ctx_timing(kp_ctx* ctx, int enable);
kp_status kp_ctx_timing_read(kp_ctx* ctx, double* total_ms, int64_t* launches);

/* Truncated multiplication (Section 3 names efficient truncation among the
   requirements of a series multiplier).  While a truncation is set, Laurent
   products computed with this context (kp_mul_laurent and the from-exponents
   calls, also inside batches, at the time they are queued) keep only the
   terms whose weighted degree sum_v weights[v] * e_v is at most max_degree;
   variables from nvars on have weight 0.  A pair of terms over the limit is
   never generated in hash mode and is sent to the discard slot in dense mode
   (the degree is linear, so the pair test deg_a + deg_b <= max_degree is
   exact).  weights: nvars (1..KP_MAX_VARS) values in [-2^15, 2^15].  Every
   factor term's weighted degree must lie in [-2^30, 2^30], else the multiply
   reports KP_E_RANGE.  Poisson products reject a set truncation (KP_E_ARG).
   kp_ctx_clear_truncation removes it.  Workspace sizes (kp_mul_bound, the
   plan calls) include the truncation tables while one is set. */
kp_status kp_ctx_set_truncation(kp_ctx* ctx, int32_t nvars, const int32_t* weights,
                                int64_t max_degree);
/* Truncation of Poisson products by the order of the Fourier harmonics
   (another criterion Section 3 names).  While set, Poisson products computed
   with this context keep only the terms whose weighted harmonic order
   sum_k weights[k] * |j_k| is at most max_order (trigonometric variables from
   ny on have weight 0).  When every factor multiplier lies in [-127, 127],
   each pair's two pieces have their orders computed from the factors'
   multipliers and a piece over the limit is never formed.  Otherwise a pair
   whose factor orders differ by more than max_order makes no piece (both of
   its pieces' orders are at least that difference), the other pieces are
   formed, and the terms over the limit are dropped where the sums are
   compacted.  Either way the result is the same.  Such products run in hash mode in
   the grouped layout (the automatic mode; KP_DENSE is KP_E_MODE).  weights: ny
   (1..KP_MAX_VARS) values in [0, 2^15].  Laurent products are unaffected.
   kp_ctx_clear_truncation removes it (and the Laurent one). */
kp_status kp_ctx_set_harmonic_truncation(kp_ctx* ctx, int32_t ny, const int32_t* weights,
                                         int64_t max_order);
kp_status kp_ctx_clear_truncation(kp_ctx* ctx);

/* Hash-table statistics (Section 3.2: open addressing with linear probing).
   While enabled, every hash-mode multiply adds to two device counters in the
   context's status block: the number of term products inserted (nonzero
   ones) and the number of slots visited beyond each product's home slot.
   Their ratio is the mean extra probe length the load factor buys.
   kp_ctx_hash_stats_read synchronises `stream`, returns both counts and, for
   the bucketed table, the products sent to its overflow table (overflows may
   be null), and clears them.  Enabling costs one atomic pair per wavefront per launch.
   Disabled by default. */
kp_status kp_ctx_hash_stats(kp_ctx* ctx, int enable);
kp_status kp_ctx_hash_stats_read(kp_ctx* ctx, hipStream_t stream, int64_t* inserts,
                                 int64_t* extra_probes, int64_t* overflows);

/* Measured denominator of the dense window kernel's roofline (Section 3.1:
   the dense accumulation is one read-modify-write of a counter per term
   product, held in LDS).  Times LDS atomic adds on every compute unit, one
   1024-thread workgroup with a 128 KiB array per unit: pattern 0 gives each
   wavefront 64 consecutive 8-byte counters (no bank conflicts), pattern 1
   pseudo-random 8-byte counters, patterns 2 and 3 the same with 4-byte
   counters; pattern 4 times the 128-bit accumulation of KP_I128 at random
   slots (a returning add on the low word, then the carry into the high
   word) and counts one such pair as one add.  Writes the device-wide rate in
   adds per second to *adds_per_second.  Runs twice (the first run warms up) and synchronises
   `stream`.  Touches no caller memory; KP_E_ARG for another pattern. */
kp_status kp_probe_lds_atomic(kp_ctx* ctx, int pattern, double* adds_per_second,
                              hipStream_t stream);

/*
 * Per-variable minimum and maximum of an int32 [n][nvars] device array, into
 * the device array out[2*nvars] = {min_0..min_{nvars-1}, max_0..max_{nvars-1}}.
 * With n == 0 the result is min = 0, max = -1 for every variable (an empty
 * box, which kp_layout_product turns into an empty product).  Used to
 * derive the factor boxes of a layout (Section 2, e_min / e_max).
 */
kp_status kp_minmax(kp_ctx* ctx, int64_t n, int32_t nvars, const int32_t* vals, int32_t* out,
                    unsigned flags, hipStream_t stream);

/*
 * Host only.  Builds the product layout from the factors' boxes (Section 2,
 * the definitions of w_k, c and chi).  amin..bmax: host int32[nx];
 * ha, hb: host int32[ny] (maximum |multiplier| per trig variable; may be null
 * when ny == 0).  An empty factor is passed as min > max and makes the
 * product empty (nkeys = 0).  Returns KP_E_CODE_OVERFLOW when the key space
 * reaches 2^62.
 */
kp_status kp_layout_product(int32_t nx, int32_t ny, const int32_t* amin, const int32_t* amax,
                            const int32_t* bmin, const int32_t* bmax, const int32_t* ha,
                            const int32_t* hb, kp_layout* out);

/*
 * Kronecker encode of one factor (Section 2, c(e) = c.e - chi; which = 0 for
 * factor A, 1 for factor B).  Device in: x_exps int32[n][nx]; for Poisson
 * (ny > 0) also y_mult int32[n][ny] and is_sin uint8[n] (may be null when
 * ny == 0).  Device out: xcodes int64[n]; for Poisson ycodes int64[n]
 * (signed balanced code).  A term outside the factor box latches KP_E_RANGE;
 * a non-canonical Poisson term latches KP_E_NONCANONICAL.
 */
kp_status kp_encode(kp_ctx* ctx, const kp_layout* layout, int which, int64_t n,
                    const int32_t* x_exps, const int32_t* y_mult, const uint8_t* is_sin,
                    int64_t* xcodes, int64_t* ycodes, unsigned flags, hipStream_t stream);

/*
 * Host only.  Sizes the caller must provide for a multiply: the resolved
 * accumulator mode, an upper bound on the number of result terms
 * (min(na*nb*(poisson ? 2 : 1), nkeys)) and the workspace bytes.
 * KP_E_MODE if KP_DENSE is asked for a key space too large for dense mode;
 * KP_E_DTYPE for an integer Poisson product.
 */
kp_status kp_mul_bound(kp_ctx* ctx, const kp_layout* layout, int poisson, kp_dtype dtype,
                       kp_mode mode, int64_t na, int64_t nb, kp_mode* resolved,
                       int64_t* max_out_terms, size_t* workspace_bytes);

/*
 * Product of two Laurent polynomials given as Kronecker-coded sparse vectors
 * (Section 3: the univariate schoolbook product of the coded factors).
 * Device in: a_codes int64[na], a_coef (int64 or double)[na], same for B;
 * unsorted input and repeated codes are accepted (the product is bilinear).
 * Device out: out_codes int64[out_cap] (product codes in [0, nkeys)),
 * out_coef[out_cap], out_n int64[1] = number of terms written.  Terms whose
 * coefficient is exactly zero are dropped.  Dense mode writes ascending
 * codes; hash mode's order is unspecified.  int64 arithmetic wraps modulo
 * 2^64.  workspace: device, >= the kp_mul_bound figure, caller-owned,
 * contents undefined afterwards.
 */
kp_status kp_mul_laurent(kp_ctx* ctx, const kp_layout* layout, kp_dtype dtype, kp_mode mode,
                         unsigned flags, const int64_t* a_codes, const void* a_coef, int64_t na,
                         const int64_t* b_codes, const void* b_coef, int64_t nb,
                         int64_t* out_codes, void* out_coef, int64_t out_cap, int64_t* out_n,
                         void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Allocation-free kp_mul_laurent, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The same product with the same arguments, except that
 * the workspace is a scratch array the library keeps in device memory,
 * KP_SCRATCH_BYTES (64 MiB) per GPU, reserved when the library's code is
 * loaded on that GPU and held until the process ends; the call allocates no
 * device memory and creates no events.  KP_E_WORKSPACE (nothing queued) when
 * the product's workspace (kp_mul_bound) is larger than the scratch array;
 * KP_E_DEVICE when the array's address could not be found at context
 * creation.  Every call on one GPU uses that GPU's one array, which keeps the
 * last call's contents (each call initialises what it needs): calls on one
 * stream are ordered and safe, calls that overlap on one GPU (different
 * streams, or asynchronous calls on different streams) race and give
 * undefined results.
 */
#define KP_SCRATCH_BYTES ((size_t)64 << 20)
kp_status kp_mul_laurent_noalloc(kp_ctx* ctx, const kp_layout* layout, kp_dtype dtype,
                                 kp_mode mode, unsigned flags, const int64_t* a_codes,
                                 const void* a_coef, int64_t na, const int64_t* b_codes,
                                 const void* b_coef, int64_t nb, int64_t* out_codes,
                                 void* out_coef, int64_t out_cap, int64_t* out_n,
                                 hipStream_t stream);

/*
 * Product of two Poisson series (Section 1, eq. ps_def) in canonical form.
 * Device in per factor: x codes int64[n], signed trig codes int64[n],
 * is_sin uint8[n], coefficients double[n].  Every pair contributes
 * 1/2 * ca * cb to cos/sin of the difference and of the sum of its arguments
 * (eq. werner with the factor 1/2), folded to canonical form; a sine of the
 * zero vector is dropped.  Device out: keys int64 (2*(kx + Wx*|ky|) + is_sin),
 * coefficients double, out_n as for kp_mul_laurent.  fp64 only.
 */
kp_status kp_mul_poisson(kp_ctx* ctx, const kp_layout* layout, kp_mode mode, unsigned flags,
                         const int64_t* a_x, const int64_t* a_y, const uint8_t* a_sin,
                         const double* a_coef, int64_t na, const int64_t* b_x,
                         const int64_t* b_y, const uint8_t* b_sin, const double* b_coef,
                         int64_t nb, int64_t* out_keys, double* out_coef, int64_t out_cap,
                         int64_t* out_n, void* workspace, size_t workspace_bytes,
                         hipStream_t stream);

/*
 * Decode product codes back to multi-indices (the inverse of the code map of
 * Section 2).  Device in: codes int64[n] (Laurent product codes, or Poisson
 * keys when poisson != 0).  Device out: x_exps int32[n][nx]; for Poisson
 * y_mult int32[n][ny] (canonical) and is_sin uint8[n].  A code outside
 * [0, nkeys) latches KP_E_RANGE.
 */
kp_status kp_decode(kp_ctx* ctx, const kp_layout* layout, int poisson, int64_t n,
                    const int64_t* codes, int32_t* x_exps, int32_t* y_mult, uint8_t* is_sin,
                    unsigned flags, hipStream_t stream);

/*
 * Whole products from exponents, in two calls (Sections 2 and 3: the code
 * map from the factors' boxes, then the product of the coded factors, then
 * the inverse map).  The plan call finds both factors' per-variable boxes in
 * one kernel launch and waits for them (the kernel hands them over through
 * a pinned host-coherent mailbox of the context, no stream synchronisation;
 * serialised per context), then fills the product layout, the resolved
 * mode, a bound on the result terms and the workspace bytes.  The multiply
 * call queues encode, multiply and decode on `stream`; the decode reads the
 * result count on the device.  The result lands in out_exps
 * int32[out_cap][nvars] and out_coef[out_cap] (int64 or double); *out_n
 * (device) is the number of terms, or -status on error (as for
 * kp_mul_laurent, including errors of the encode, e.g. KP_E_RANGE for
 * exponents outside the planned boxes).  With KP_FLAG_ASYNC the call
 * returns once the work is queued and n_host is unused; without it the call
 * waits for the count (through the mailbox), stores it in *n_host (when not
 * null) and returns any error, read and cleared as by kp_ctx_check.
 * Terms whose coefficient is exactly zero are dropped; order as for
 * kp_mul_laurent.  Device in: a_exps int32[na][nvars], a_coef[na], same for
 * B.  workspace: device, >= the planned bytes, caller-owned, contents
 * undefined afterwards.  KP_E_WORKSPACE if it is smaller; KP_E_CODE_OVERFLOW
 * (plan) when the product's codes would not fit in 62 bits.
 */
kp_status kp_plan_laurent(kp_ctx* ctx, int32_t nvars, kp_dtype dtype, kp_mode mode,
                          const int32_t* a_exps, int64_t na, const int32_t* b_exps, int64_t nb,
                          kp_layout* layout, kp_mode* resolved, int64_t* max_out_terms,
                          size_t* workspace_bytes, hipStream_t stream);
kp_status kp_mul_laurent_exps(kp_ctx* ctx, const kp_layout* layout, kp_dtype dtype, kp_mode mode,
                              unsigned flags, const int32_t* a_exps, const void* a_coef, int64_t na,
                              const int32_t* b_exps, const void* b_coef, int64_t nb,
                              int32_t* out_exps, void* out_coef, int64_t out_cap, int64_t* out_n,
                              int64_t* n_host, void* workspace, size_t workspace_bytes,
                              hipStream_t stream);

/*
 * Plan and multiply in one call, for callers that keep buffers across
 * products of similar size: the plan as kp_plan_laurent (its layout into
 * *layout), then, when out_cap and workspace_bytes cover it, the multiply as
 * kp_mul_laurent_exps.  *need_cap and *need_workspace always receive the
 * sizes this product needs; when the given ones are smaller the call returns
 * KP_E_WORKSPACE with nothing queued after the plan, and the caller may
 * continue with kp_mul_laurent_exps and the returned layout.
 */
kp_status kp_mul_laurent_auto(kp_ctx* ctx, int32_t nvars, kp_dtype dtype, kp_mode mode,
                              unsigned flags, const int32_t* a_exps, const void* a_coef, int64_t na,
                              const int32_t* b_exps, const void* b_coef, int64_t nb,
                              int32_t* out_exps, void* out_coef, int64_t out_cap, int64_t* out_n,
                              int64_t* n_host, void* workspace, size_t workspace_bytes,
                              kp_layout* layout, int64_t* need_cap, size_t* need_workspace,
                              hipStream_t stream);

/*
 * The same two calls for Poisson series in canonical form (Section 1,
 * eq. ps_def; products by eq. werner as in kp_mul_poisson).  Per factor:
 * x exponents int32[n][nx] (nx may be 0, then the x arrays may be null),
 * trigonometric multipliers int32[n][ny] (ny >= 1), is_sin uint8[n],
 * coefficients double[n].  The trigonometric half-widths of the layout are
 * the largest |multiplier| per variable of each factor.  Out: out_x
 * int32[out_cap][nx], out_y int32[out_cap][ny] (canonical: first nonzero
 * multiplier positive), out_sin uint8[out_cap], out_coef double[out_cap],
 * *out_n (device), n_host as above.  A non-canonical input term gives
 * KP_E_NONCANONICAL.
 */
kp_status kp_plan_poisson(kp_ctx* ctx, int32_t nx, int32_t ny, kp_mode mode, const int32_t* a_x,
                          const int32_t* a_y, int64_t na, const int32_t* b_x, const int32_t* b_y,
                          int64_t nb, kp_layout* layout, kp_mode* resolved,
                          int64_t* max_out_terms, size_t* workspace_bytes, hipStream_t stream);
kp_status kp_mul_poisson_exps(kp_ctx* ctx, const kp_layout* layout, kp_mode mode, unsigned flags,
                              const int32_t* a_x, const int32_t* a_y, const uint8_t* a_sin,
                              const double* a_coef, int64_t na, const int32_t* b_x,
                              const int32_t* b_y, const uint8_t* b_sin, const double* b_coef,
                              int64_t nb, int32_t* out_x, int32_t* out_y, uint8_t* out_sin,
                              double* out_coef, int64_t out_cap, int64_t* out_n, int64_t* n_host,
                              void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Batches: many products queued by one call (a systems pattern; it does not
 * change what any product computes).  A batch holds up to max_tasks
 * descriptors, each the arguments of one kp_mul_laurent or kp_mul_poisson
 * call, copied in by kp_batch_add (the layout by value; the arrays stay owned
 * by the caller and must stay valid while the batch is used).  kp_batch_add
 * runs every host check of the single call and reports its errors at once.
 *
 * kp_batch_launch queues all tasks in order on `stream` and returns without
 * synchronising; each task's out_n receives its term count or -(status).
 * With KP_BATCH_GRAPH the first launch captures the queued kernels into a
 * HIP graph and later launches replay it: the same tasks on the same arrays
 * (their contents may change between launches); capture needs a stream other
 * than the null stream.  kp_batch_add and
 * kp_batch_clear drop the graph.  kp_batch_status synchronises the stream of
 * the last launch and returns one task's count (status = its error, if any).
 * Tasks of one batch must not share workspace or output arrays.
 */
typedef enum { KP_KIND_LAURENT = 0, KP_KIND_POISSON = 1 } kp_kind;
enum { KP_BATCH_GRAPH = 2 };

typedef struct kp_mul_desc {
  kp_kind kind;
  kp_layout layout;            /* product layout (kp_layout_product)                */
  kp_dtype dtype;              /* Laurent coefficient type; Poisson is fp64         */
  kp_mode mode;
  const int64_t* a_codes;      /* device: Laurent codes, or Poisson x codes [na]    */
  const int64_t* a_y;          /* device: Poisson trig codes [na] (else null)       */
  const uint8_t* a_sin;        /* device: Poisson sine flags [na] (else null)       */
  const void* a_coef;          /* device: coefficients [na]                         */
  int64_t na;
  const int64_t* b_codes;
  const int64_t* b_y;
  const uint8_t* b_sin;
  const void* b_coef;
  int64_t nb;
  int64_t* out_codes;          /* device: result codes / keys [out_cap]             */
  void* out_coef;              /* device: result coefficients [out_cap]             */
  int64_t out_cap;
  int64_t* out_n;              /* device: int64[1]                                  */
  void* workspace;             /* device: kp_mul_bound's workspace_bytes            */
  size_t workspace_bytes;
} kp_mul_desc;

typedef struct kp_batch kp_batch;
kp_status kp_batch_create(kp_ctx* ctx, int64_t max_tasks, kp_batch** out);
kp_status kp_batch_destroy(kp_batch* batch);
kp_status kp_batch_add(kp_batch* batch, const kp_mul_desc* desc, int64_t* task_id);
kp_status kp_batch_clear(kp_batch* batch);
kp_status kp_batch_launch(kp_batch* batch, unsigned flags, hipStream_t stream);
kp_status kp_batch_status(kp_batch* batch, int64_t task_id, int64_t* n_out);

/*
 * Packed batches: many whole Laurent products of uneven sizes in one fixed
 * sequence of persistent launches (a systems pattern; each product is the
 * schoolbook sum of Section 3 over the Kronecker codes of Section 2, the same
 * set of terms as kp_mul_laurent_exps gives).  The products' descriptions sit
 * in a device task table; each stage is one launch of a fixed grid whose
 * workgroups walk the work of every task (encode both factors and clear the
 * accumulator; form every pair's product and add it at its code; compact the
 * nonzero sums, decoding them to exponents; post the counts).  Each product
 * accumulates in device memory of its own: one word per code when the key
 * space is at most twice the size of the hash table it would otherwise get
 * (Section 3.1's dense array), else an open-addressing hash table of at least
 * twice the result bound, compare-and-swap on the key and atomic add on the
 * coefficient (Section 3.2).  Meant for many small products, whose cost per
 * call is launches and host waits; large products are better served one call
 * each.
 *
 * kp_pack_create: a pack for up to max_tasks (1..4096) products; it owns a
 *   device task table and pinned host memory for the boxes and counts.
 * kp_pack_plan: tasks[0..n) (device arrays: exponents int32 [n][nvars],
 *   coefficients int64 or double; KP_E_DTYPE otherwise) are copied in; one
 *   launch takes every factor's box and one host wait brings them back; each
 *   product's layout (Section 2, KP_E_CODE_OVERFLOW) and result bound
 *   min(codes, na nb) follow.  out_cap[k] receives task k's bound,
 *   *arena_bytes the device memory kp_pack_run needs.
 * kp_pack_run: queues the products on `stream` and returns: task k's terms
 *   go to out_exps[k] (int32 [out_cap[k]][nvars]) and out_coef[k]
 *   ([out_cap[k]], the task's type), in unspecified order.  `arena` is
 *   caller-owned device memory of at least *arena_bytes.  With KP_PACK_GRAPH
 *   the upload of the table and the four launches are captured into a HIP
 *   graph at the first such run and replayed by every later one (any
 *   products: the kernels read them from the table); capture needs a stream
 *   other than the null stream.
 * kp_pack_wait: waits for the counts of the last run (one host wait for the
 *   whole batch); n_out[k] is task k's number of terms, or -(status) after a
 *   device error (the call then returns that status).  kp_pack_query sets
 *   *done without waiting.
 * A pack runs one batch at a time: plan and run refuse while a run has not
 * been waited for.  The caller keeps the arrays valid until the wait.
 */
typedef struct kp_pack kp_pack;
enum { KP_PACK_GRAPH = 4 };

typedef struct kp_pack_task {
  int32_t nvars;               /* 1..KP_MAX_VARS                                    */
  kp_dtype dtype;              /* KP_I64 or KP_F64                                  */
  const int32_t* a_exps;       /* device [na][nvars]                                */
  const void* a_coef;          /* device [na]                                       */
  int64_t na;                  /* < 2^31                                            */
  const int32_t* b_exps;
  const void* b_coef;
  int64_t nb;
} kp_pack_task;

kp_status kp_pack_create(kp_ctx* ctx, int32_t max_tasks, kp_pack** out);
kp_status kp_pack_destroy(kp_pack* pack);
kp_status kp_pack_plan(kp_pack* pack, const kp_pack_task* tasks, int32_t n, int64_t* out_cap,
                       size_t* arena_bytes, hipStream_t stream);
kp_status kp_pack_run(kp_pack* pack, int32_t* const* out_exps, void* const* out_coef, void* arena,
                      size_t arena_bytes, unsigned flags, hipStream_t stream);
kp_status kp_pack_wait(kp_pack* pack, int64_t* n_out);
kp_status kp_pack_query(kp_pack* pack, int32_t* done);

/*
 * Host-memory twins of kp_encode / kp_decode, running the same per-term code
 * map on the CPU (for callers without a device and for checking tables).
 * Errors are returned directly.
 */
kp_status kp_encode_host(const kp_layout* layout, int which, int64_t n, const int32_t* x_exps,
                         const int32_t* y_mult, const uint8_t* is_sin, int64_t* xcodes,
                         int64_t* ycodes);
kp_status kp_decode_host(const kp_layout* layout, int poisson, int64_t n, const int64_t* codes,
                         int32_t* x_exps, int32_t* y_mult, uint8_t* is_sin);

#ifdef __cplusplus
}
#endif

#endif /* KP_H */
