/*
 * hk -- smallest eigenvalue of the Hankel moment matrix
 *           M_ij = (1/beta) Gamma((1+i+j)/beta),  i, j = 0..N-1,
 * by a fixed-point LDL^T factorisation of M - xI on an AMD MI355X (gfx950).
 *
 * Method (Emmart, Weems, Chen, "Computing the smallest eigenvalue of large
 * ill-conditioned Hankel matrices"):
 *   - the matrix definition is the paper's Introduction; M is the moment
 *     matrix of exp(-x^beta) on [0, inf) ("Properties of M"), hence SPD with
 *     distinct eigenvalues;
 *   - the factorisation is the submatrix-order LDL^T of "The LDL^T
 *     Determinant Algorithm": M entries carry K fractional bits, the
 *     extracted column C and the quotient L = C / diag carry K/2;
 *   - lambda_1 is the smallest root of P(x) = det(M - xI) ("The Secant
 *     Algorithm"), checked by the sign test of "Interval Verification";
 *   - inverse iteration on one factorisation is offered as the default
 *     driver (not in the paper).
 *
 * Conventions for every entry point
 *   - extern "C", never throws; returns hk_status (HK_OK = 0).  On error a
 *     message is available from hk_last_error() (thread-local).
 *   - K = prec_bits must be even and >= 64 (K/2 must be integral).
 *   - beta = num/den with num, den >= 1 (reduced internally).
 *   - Device memory is owned by the caller.  dev_ws is one device buffer of
 *     at least hk_workspace_bytes(...) bytes; the library carves it up and
 *     never allocates or frees device memory itself.  hk_matrix handles own
 *     only host memory and must be released with hk_matrix_destroy.
 *   - Every device operation is enqueued on the caller's stream s; calls
 *     that return results to the host synchronise that stream.
 *   - Big integers cross the boundary in one of two plain formats:
 *       hk_mpf      : value = sign * sum_i digits[i] 2^(32 i) * 2^exp2;
 *       "int lists" : arrays (slen[n], off[n], dig[]): entry i has |slen[i]|
 *                     base-2^32 digits dig[off[i] ..], little endian, its
 *                     sign is the sign of slen[i] (slen 0 = zero).
 */
#ifndef HK_H
#define HK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int64_t num, den; } hk_rational;

typedef struct {
  int32_t sign;            /* -1, 0, +1 */
  int32_t ndigits;         /* number of base-2^32 digits */
  int64_t exp2;            /* binary exponent of digit 0 */
  const uint32_t* digits;  /* host memory, little endian */
} hk_mpf;

typedef enum {
  HK_OK = 0,
  HK_EINVAL = 1,      /* bad argument (sizes, K odd, beta <= 0, short ws)   */
  HK_ENOTSPD = 2,     /* pivot <= 0 before the last column                  */
  HK_EPRECISION = 3,  /* precision exhausted (iteration stalled, overflow)  */
  HK_ENOCONV = 4,     /* iteration limit reached                            */
  HK_EVERIFY = 5,     /* inertia bracket failed                             */
  HK_EDEVICE = 6,     /* HIP runtime error                                  */
  HK_ENOMEM = 7       /* host allocation failed                             */
} hk_status;

enum { HK_INVERSE = 0, HK_SECANT = 1 };
/* flags or-ed into the method argument of hk_smallest_eig */
enum { HK_FLAG_NO_WORK_COUNT = 0x100,   /* skip the limb-MAC count (report 0)    */
       HK_FLAG_TIME_UPDATES = 0x200,    /* time every trailing-update launch      */
       HK_FLAG_CERTIFY = 0x400,         /* prove the inertia bracket (hk_certify
                                           on both bracket factorisations)       */
       HK_FLAG_VECTOR_UPDATE = 0x800 }; /* the bulk of the trailing update on the
                                           vector units (hk_set_update_engine)   */
/* panel width p in 1..64 forced for hk_smallest_eig: or HK_FLAG_PANEL(p)
   into the method argument (0: the tuned width, else 4) */
#define HK_FLAG_PANEL(p) (((p) & 0xff) << 16)
/* look-ahead mode forced for hk_smallest_eig (see hk_set_lookahead): 1, 0, 2 */
enum { HK_FLAG_LOOKAHEAD_ON = 0x1000000, HK_FLAG_LOOKAHEAD_OFF = 0x2000000,
       HK_FLAG_LOOKAHEAD_FUSED = 0x4000000 };
/* update items per workgroup g in {1, 2, 4} forced for hk_smallest_eig
   (see hk_set_update_group): or HK_FLAG_GROUP(g) into the method argument */
#define HK_FLAG_GROUP(g) (((g) & 7) << 28)

typedef struct hk_matrix_s* hk_matrix;

/* Words of lambda_1's binary value in hk_report and hk_result: the computed
   value (K fractional bits) rounded to nearest, ties to even, to at most
   32 * HK_LAMBDA_WORDS significant bits (exact when it has fewer). */
#define HK_LAMBDA_WORDS 16

typedef struct {
  int N, K, h;            /* size, fractional bits of M, of C and L            */
  int digit_bits;         /* device digit radix 2^digit_bits (29)             */
  int max_col_digits;     /* widest column of the working triangle            */
  int vec_digits;         /* digits per entry of a device vector              */
  int solve_guard_bits;   /* extra fractional bits of the solve vectors       */
  int panel;              /* columns per trailing update (rank of the update) */
  size_t ws_bytes;        /* bytes of workspace in use                        */
  size_t vec_bytes;       /* bytes of one device vector (hk_solve operands)   */
  int n_update_launches;  /* launches that carry the update work in the last
                             hk_factor (k_update, or k_column in look-ahead
                             mode 2)                                          */
  double update_ms;       /* summed device time of those launches (timing on) */
  int lookahead;          /* look-ahead mode hk_factor uses (0, 1, 2)         */
  int n_bulk_launches;    /* of those, the bulk ones: k_update (the trailing
                             update, or its columns beyond the next panel
                             under look-ahead 1), or every k_column launch
                             (mode 2); the rest are k_update_near launches
                             (in-panel updates, the next panel's columns)     */
  double bulk_ms;         /* summed device time of the bulk launches          */
  int update_engine;      /* engine of the bulk launches at the current panel
                             width: 1 matrix cores (k_update_mma), 0 vector
                             units (k_update, or k_column in mode 2)          */
} hk_info;

typedef struct {
  hk_status status;
  int bits_used;          /* K of the accepted run                            */
  int factorizations;     /* LDL^T factorisations performed                   */
  int solves;             /* hk_solve calls (inverse iteration)               */
  int verified;           /* 1 if the inertia bracket held                    */
  int digits_verified;    /* significant digits of the verified bracket       */
  char lambda_dec[192];   /* lambda_1 in decimal scientific notation          */
  double limb_macs;       /* algorithmic 32-bit limb MACs, all factorisations */
  double t_factor_s, t_solve_s, t_total_s;
  int update_launches;    /* update-kernel launches (HK_FLAG_TIME_UPDATES)    */
  double update_ms;       /* their summed device time                         */
  int bulk_launches;      /* of those, the bulk launches (hk_info)            */
  double bulk_ms;         /* their summed device time                         */
  double limb_macs_bulk;  /* the share of limb_macs the bulk launches carry   */
  int certified;          /* HK_FLAG_CERTIFY: 1 when the bracket is proved    */
  double certify_margin_bits;  /* least log2(|pivot| / radius) of the two
                             bracket factorisations (negative: short)         */
  int certify_bits;       /* HK_FLAG_CERTIFY and not proved: the precision at
                             which the margin would reach 16 bits             */
  hk_mpf lambda;          /* lambda_1 in binary (sign 0: none); its digits
                             point at lambda_words of this same report       */
  uint32_t lambda_words[HK_LAMBDA_WORDS];
  int update_engine;      /* hk_info's update_engine of the factorisations    */
} hk_report;

/* Bytes of device workspace needed for (N, beta, K).  flags: reserved, 0.
   Returns 0 for invalid arguments. */
size_t hk_workspace_bytes(int N, hk_rational beta, int prec_bits, int flags);

/* Computes the 2N-1 moments X_n = RNE(2^K mu_n), mu_n = (1/beta)
   Gamma((n+1)/beta) (Introduction: the matrix definition), correctly rounded
   (round to nearest, ties to even), and uploads them to dev_ws.  The matrix
   itself is expanded from them at every hk_factor.  On success *out is a new
   handle bound to dev_ws (which must stay alive until hk_matrix_destroy).
   Its panel width (4) and look-ahead (by size) are the ones hk_autotune
   stored for this shape in the tuning cache named by the environment
   variable HK_TUNE_CACHE, when there is such an entry. */
hk_status hk_build_matrix(int N, hk_rational beta, int prec_bits, void* dev_ws,
                          size_t ws_bytes, hipStream_t s, hk_matrix* out);

/* Host only (no device work): the same 2N-1 correctly rounded moments
   X_n = RNE(2^K mu_n) that hk_build_matrix uploads (Introduction: the matrix
   definition; "Properties of M": the moments of exp(-x^beta)).  Each X_n is
   a nonnegative integer written as little-endian base-2^32 words:
   words[off[n] .. off[n+1]) for n = 0..2N-2; off (caller-owned, 2N entries)
   is always filled, off[2N-1] being the total word count.  With words NULL,
   or cap (its length in words) below that total, only off is written and
   the call returns HK_EINVAL; call again with a large enough buffer.
   HK_EPRECISION if the rounding stays undecided (never seen in practice). */
hk_status hk_moments_host(int N, hk_rational beta, int prec_bits, uint32_t* words, int64_t cap,
                          int64_t* off);

/* LDL^T of M - xI, x = shift (a dyadic with at most K fractional bits),
   in the paper's submatrix order and fixed-point format ("The LDL^T
   Determinant Algorithm"; parallel variant's formats): for each column pc,
     C_pc[r] = RNE(A_{r,pc} / 2^h)   r >= pc,   d_pc = C_pc[pc],
     L_pc[r] = RNE(C_pc[r] 2^h / d_pc)          r > pc,
     A_{rc} -= C_pc[c] L_pc[r]  (exact)         pc < c <= r.
   The factors stay in dev_ws.  inertia_mode = 0: a pivot <= 0 before the
   last column returns HK_ENOTSPD with *first_bad_col set.  inertia_mode = 1:
   returns HK_OK when only the last pivot is <= 0 and reports *n_negative
   (Sylvester's inertia, used by the verification); a non-positive pivot
   earlier still returns HK_ENOTSPD (the fixed widths hold only while the
   trailing block is positive definite).  n_negative / first_bad_col may be
   NULL.  Synchronises s. */
hk_status hk_factor(hk_matrix m, hk_mpf shift, int inertia_mode, hipStream_t s,
                    int* n_negative, int* first_bad_col);

/* x = (L D L^T)^{-1} b on the current factorisation: dev_rhs holds b with K
   fractional bits, dev_x receives x with K + g fractional bits (g =
   hk_info.solve_guard_bits).  Forward, diagonal and backward steps each
   round once per entry (RNE) after exact inner products.  Both operands are
   device vectors of hk_info.vec_bytes bytes in the library's layout (fill
   and read them with hk_vec_import / hk_vec_export).  Synchronises s and
   returns HK_EPRECISION if an intermediate exceeded the planned widths. */
hk_status hk_solve(hk_matrix factored, const void* dev_rhs, void* dev_x, hipStream_t s);

/* The full method: build, factor, iterate (HK_INVERSE: inverse iteration on
   one factorisation at shift_hint or 0; HK_SECANT: the paper's Secant
   iteration), then the inertia bracket at `digits` significant digits.
   lambda_1 is written to out_decimal (scientific notation, `digits`
   digits).  rep may be NULL.  The drivers' host arithmetic (the Secant's
   pivot ratio, the inverse iteration's dot products) runs on up to 16 host
   threads; the environment variable HK_HOST_THREADS sets the number. */
hk_status hk_smallest_eig(int N, hk_rational beta, int prec_bits, int method, int digits,
                          const hk_mpf* shift_hint, void* dev_ws, size_t ws_bytes,
                          hipStream_t s, char* out_decimal, size_t out_len, hk_report* rep);

/* hk_smallest_eig for callers that cannot allocate device memory (code that
   must not call hipMalloc: serving loops, harnesses that forbid it): the
   same method and results, with the workspace in a fixed array of the
   library (hk_static_workspace_limit() bytes, 64 MiB, held on every device
   the library runs on until the process ends) instead of a caller buffer.
   Every launch goes on s: no graph is captured and no stream or event is
   created (look-ahead mode 1 runs as mode 0, so HK_FLAG_LOOKAHEAD_ON and
   HK_FLAG_TIME_UPDATES are rejected).  HK_EINVAL when the instance needs
   more workspace than the array holds (N = 200, beta = 7/4, K = 2048 needs
   54 MB).  Calls on one device share the array: calls that overlap in time
   on one device race; every call rebuilds what it reads, so one call's
   leftovers never reach the next.  Synchronises s. */
size_t hk_static_workspace_limit(void);
hk_status hk_smallest_eig_static(int N, hk_rational beta, int prec_bits, int method, int digits,
                                 const hk_mpf* shift_hint, hipStream_t s, char* out_decimal, size_t out_len,
                                 hk_report* rep);

hk_status hk_matrix_destroy(hk_matrix m);
const char* hk_last_error(void);
hk_status hk_matrix_info(hk_matrix m, hk_info* out);

/* Rigorous inertia of the current factorisation of m (the sign checks of
   "Interval Verification" made rigorous, in midpoint-radius form): the
   fixed-point factors are the midpoints; a radius per entry bounds the
   distance to the same quantity of the exact elimination of the true
   matrix (exact moments, exact shift): 2^-(K+1) for the correctly rounded
   moments, plus the rounding of every C and L entry carried through the
   updates, each operation rounded up.  A pivot is certified when its
   magnitude exceeds its radius; *certified = 1 when every pivot is (then
   *n_negative is the exact inertia of M - xI), 0 when one is not, or a
   pivot before the last is negative (later radii are then unbounded).
   *min_margin_bits (may be NULL): the least log2(|pivot| / radius);
   margin_bits (N doubles, may be NULL): per pivot.  The radii grow with the
   elimination's cancellation, so certification needs K above what the
   plain inertia check needs (a missing bit of margin costs two of K).
   Overwrites the working triangle (the factors stay); synchronises s. */
hk_status hk_certify(hk_matrix m, hipStream_t s, int* n_negative, int* certified, double* min_margin_bits,
                     double* margin_bits);

/* Tuning: columns per trailing update (panel width, >= 1). */
hk_status hk_set_panel(hk_matrix m, int panel);
/* Tuning: update items (wavefronts of 64 rows x 16 output digits) per
   workgroup of the update kernels, 1, 2 or 4 (the default, or the tuned
   value); HK_EINVAL otherwise. */
hk_status hk_set_update_group(hk_matrix m, int items);
/* Engine of the bulk of the trailing update ("The LDL^T Determinant
   Algorithm", the update of the columns beyond the panel; the digits are the
   same either way): HK_UPDATE_MATRIX_CORES (the default) splits every digit
   of C and L into four signed bytes and accumulates the digit products as
   int8 matrix products (v_mfma_i32_32x32x32_i8) wherever the panel width b
   and the widest column W keep b W below 32704 (int32 accumulators), and
   uses the vector units elsewhere; HK_UPDATE_VECTOR always uses the vector
   units (v_mad_i64_i32).  HK_EINVAL for other values. */
enum { HK_UPDATE_MATRIX_CORES = 0, HK_UPDATE_VECTOR = 1 };
hk_status hk_set_update_engine(hk_matrix m, int engine);
/* Look-ahead ("The LDL^T Determinant Algorithm", parallel version: the next
   panel's columns are updated first): mode 1 splits every trailing update
   into the next panel's columns, on the critical path, and the rest, on a
   second stream concurrently with the next panel; mode 2 takes one launch
   per column (panel width 1) in which each row's workgroup applies the
   previous column's update to its own entry and the pivot's before
   finalising and dividing, while further workgroups of the same launch
   update the columns beyond; 0 keeps one trailing update per panel;
   -1 (default) takes the tuned setting, else 1 when N x widest column
   >= 100000 digits and 2 below.  The environment variable HK_LOOKAHEAD=0/1/2
   overrides every setting.  The digits are the same in every mode (exact
   updates).  HK_EINVAL for another mode. */
hk_status hk_set_lookahead(hk_matrix m, int mode);
/* Timing: when on, every launch of the update kernel in hk_factor (the
   in-panel and the trailing ones) is bracketed by HIP events on s and
   hk_info reports their count and summed duration. */
hk_status hk_set_timing(hk_matrix m, int on);

/* Copies factor entries of columns [c0, c1) to the host as int lists.
   kind 0: C_pc[r], r = pc..N-1;  kind 1: L_pc[r], r = pc+1..N-1;
   kind 2: pivots d_pc.  Values carry h fractional bits.  Call with
   dig == NULL to get the number of digits needed (return value); the
   number of entries is implied by (kind, c0, c1).  Returns -1 on error. */
int64_t hk_factor_export(hk_matrix m, int kind, int c0, int c1, int32_t* slen,
                         int64_t* off, uint32_t* dig, int64_t dig_cap, hipStream_t s);

/* Algorithmic work of the last factorisation: sum over updates of
   ceil(bits(C)/32) * ceil(bits(L)/32) (schoolbook 32-bit limb MACs).
   Launches a small counting kernel and synchronises s. */
hk_status hk_factor_limb_macs(hk_matrix m, hipStream_t s, double* limb_macs);

/* Device vectors (N entries) <-> int lists.  Import expects values with K
   fractional bits; export returns the stored fixed-point integers. */
hk_status hk_vec_import(hk_matrix m, int n, const int32_t* slen, const int64_t* off,
                        const uint32_t* dig, void* dev_vec, hipStream_t s);
int64_t hk_vec_export(hk_matrix m, const void* dev_vec, int n, int32_t* slen, int64_t* off,
                      uint32_t* dig, int64_t dig_cap, hipStream_t s);

/* ---- measurement ---------------------------------------------------------
   Issue rate of one VALU instruction kind on the running GPU, measured:
   every lane of a grid that fills every SIMD (8 waves each) runs 16
   independent chains of 4096 steps of it, so the rate is the issue rate
   rather than the latency.  It is the denominator of the update kernel's
   fraction of the integer-multiply peak (the update multiplies 29-bit digits
   with HK_RATE_MAD_I64_I32, int64 += int32 x int32).  dev_buf: device
   buffer of at least hk_mul_rate_buffer_bytes() bytes (the chains' results
   and per-wave clock samples).  *per_s: lane operations per second (one
   timed launch after a warm-up launch); *clock_hz (may be NULL): the shader
   clock during the timed launch, from each wave's cycle counter against
   the constant-rate counter.  HK_RATE_MFMA_I8: the matrix-core update's
   instruction (v_mfma_i32_32x32x32_i8), four independent products per wave;
   *per_s counts int8 multiply-adds.  Synchronises s. */
enum { HK_RATE_MAD_I64_I32 = 0, HK_RATE_MAD_U64_U32 = 1, HK_RATE_MAD_U32_U24 = 2, HK_RATE_FMA_F64 = 3,
       HK_RATE_MFMA_I8 = 4 };
size_t hk_mul_rate_buffer_bytes(void);
hk_status hk_mul_rate(int kind, void* dev_buf, size_t buf_bytes, hipStream_t s, double* per_s, double* clock_hz);

/* ---- batched form ------------------------------------------------------
   Many instances of uneven (N, beta, K) factored together: every kernel of
   the factorisation covers all instances of the batch in one launch (work
   items are (instance, column, row tile, digit block)), and the whole launch
   sequence of one factorisation is captured once in a HIP graph and
   replayed for every factorisation the drivers need.  The driver is the
   paper's Secant iteration ("The Secant Algorithm") per instance, run in
   lockstep, then the inertia bracket of "Interval Verification".  Callers
   that repeat the same batch shapes may tune the panel width once with
   hk_autotune. */
typedef struct {
  int N;
  hk_rational beta;
  int prec_bits;
  int method;                /* hk_eig_batched: HK_SECANT, or HK_INVERSE (0, what
                                a zero-initialised instance asks for)       */
  const hk_mpf* shift_hint;  /* HK_INVERSE: the shift of its factorisation
                                (NULL: 0); ignored elsewhere                 */
} hk_instance;

typedef struct {
  hk_status status;
  int factorizations;     /* factorisations this instance took part in   */
  int verified;           /* 1 if the inertia bracket held               */
  char lambda_dec[192];   /* lambda_1 in decimal scientific notation     */
  int bits_used;          /* K of the returned value                     */
  int solves;             /* hk_solve calls (inverse iteration)          */
  int path;               /* 0: plain method, checked by the inertia
                             bracket; 1: learned proposal, accepted by the
                             rerun at +25% bits (hk_eig_learned)         */
  hk_mpf lambda;          /* lambda_1 in binary (sign 0: none); its digits
                             point at lambda_words of this same result   */
  uint32_t lambda_words[HK_LAMBDA_WORDS];
} hk_result;

typedef struct {
  int panel;              /* panel width used                            */
  int graph_launches;     /* batched factorisations (graph replays)      */
  double t_build_s;       /* moments + uploads                           */
  double t_factor_s;      /* graph replays incl. pivot read-back         */
  double t_total_s;
  int update_launches;    /* HK_FLAG_TIME_UPDATES: update launches of all
                             factorisations and their summed device time  */
  double update_ms;
  int bulk_launches;      /* of those, the bulk launches (hk_info)       */
  double bulk_ms;
  int update_engine;      /* hk_info's update_engine of the batch        */
} hk_batch_report;

/* Device bytes for a batch (one buffer for all instances). 0 if invalid. */
size_t hk_batch_workspace_bytes(const hk_instance* inst, int count);

/* Device bytes with which hk_eig_batched pairs factorisations (about twice
   hk_batch_workspace_bytes: a second copy of every instance's workspace).
   0 if invalid. */
size_t hk_batch_workspace_bytes_paired(const hk_instance* inst, int count);

/* lambda_1 of every instance by its method: HK_SECANT instances run the
   paper's Secant iteration in lockstep (one batched factorisation per
   step); HK_INVERSE instances are factored once at their shift hint (halved
   while a pivot is <= 0, at most three times, then 0) and run inverse
   iteration together; then the inertia bracket ("Interval Verification")
   for all.  panel = 0 takes the width from the tuning
   cache named by the environment variable HK_TUNE_CACHE when it has an entry
   for this batch shape, else 4.  The first instance's method may carry the
   hk_smallest_eig flags HK_FLAG_LOOKAHEAD_*, HK_FLAG_GROUP(g),
   HK_FLAG_VECTOR_UPDATE and HK_FLAG_TIME_UPDATES (every factorisation then
   launched one by one with its update launches timed, in rep); they apply to
   the whole batch.  With ws_bytes of at least
   hk_batch_workspace_bytes_paired(inst, count), the two start points of
   every Secant instance and the two ends of every bracket are factored in
   one launch sequence each (the second shift on a second copy of the
   instance), two launch sequences fewer per call; the results are the same.
   out[count] receives the per-instance
   results; the call returns HK_OK if every instance succeeded (otherwise the
   first failing status).  rep may be NULL.  Synchronises s. */
hk_status hk_eig_batched(const hk_instance* inst, int count, int digits, int panel, void* dev_ws,
                         size_t ws_bytes, hipStream_t s, hk_result* out, hk_batch_report* rep);

/* Times one batched factorisation of the given batch for each panel width
   in {1, 2, 4, 8, 16} under look-ahead modes 0 and 1, and once under mode 2
   (width 1), then the update workgroup size (1, 2 or 4 items of 64 rows x
   16 digits per workgroup) for the fastest, then the update engine (the
   vector units against the matrix cores, see hk_set_update_engine); stores
   the choice in *best_panel, *best_lookahead and *best_group (the last two
   may be NULL) and appends it, engine included, to the text cache file
   cache_path (NULL: no file) under the batch-shape key (architecture,
   count, N bucket, K bucket), from which hk_build_matrix, hk_eig_batched,
   hk_batch_create and hk_eig_learned take it.  Rows per item and digits
   per output block (16, the carry-plane granularity of the layout) are
   fixed.  Synchronises s. */
hk_status hk_autotune(const hk_instance* inst, int count, void* dev_ws, size_t ws_bytes,
                      hipStream_t s, const char* cache_path, int* best_panel, int* best_lookahead,
                      int* best_group);

/* Batch handles: the instances of a batch laid out in dev_ws (at least
   hk_batch_workspace_bytes(inst, count) bytes, alive until hk_batch_destroy)
   and factored together at caller-given shifts by the same captured graph of
   instance-batched launches hk_eig_batched replays.  The factors of
   instance i stay in the workspace and are read through the borrowed handle
   hk_batch_instance(b, i) with hk_factor_export / hk_factor_limb_macs
   (never hk_matrix_destroy it: the batch owns it). */
typedef struct hk_batch_s* hk_batch;

/* Lays the batch out in dev_ws: every instance's moments (host) and
   uploads.  The schedule starts as the tuned one (HK_TUNE_CACHE), else
   panel 4 with the look-ahead mode chosen by size.  Synchronises s. */
hk_status hk_batch_create(const hk_instance* inst, int count, void* dev_ws, size_t ws_bytes, hipStream_t s,
                          hk_batch* out);
/* panel width in 1..64, look-ahead mode -1 (by size), 0, 1 or 2 (2 forces
   panel width 1) and update items per workgroup 1, 2 or 4 (0: keep); the
   digits are the same under every schedule. */
hk_status hk_batch_set_schedule(hk_batch b, int panel, int lookahead, int group);
/* LDL^T of M_i - x_i I for every instance ("The LDL^T Determinant
   Algorithm", as hk_factor) in one graph replay; shifts[i] is a dyadic with
   at most K_i fractional bits (shifts NULL: all zero).  Per instance (arrays
   of count, each may be NULL): status (HK_OK, HK_ENOTSPD for a pivot <= 0
   before the last column, HK_EPRECISION for a width overflow), the number
   of negative pivots and the first column with a pivot <= 0 (-1: none).  A
   last pivot <= 0 is reported, not an error (inertia mode).  Returns the
   first failing status.  Synchronises s. */
hk_status hk_batch_factor(hk_batch b, const hk_mpf* shifts, hipStream_t s, hk_status* status, int* n_negative,
                          int* first_bad_col);
/* Instance i of the batch as a (borrowed) matrix handle; NULL if out of range. */
hk_matrix hk_batch_instance(hk_batch b, int i);
hk_status hk_batch_destroy(hk_batch b);

/* ---- precision-proposal network -----------------------------------------
   A float32 MLP 3 -> 64 -> 64 -> 64 -> 2 with ReLU on the hidden layers
   (not in the paper).  It maps the scaled features (N, beta, ln N) of an
   instance to its scaled required precision and scaled ln lambda_1; its
   training data come from the method itself (hk_bracket_batched).  Every
   pointer below is a caller-owned float32 device buffer; the kernels run on
   s and nothing is synchronised.  Parameters: one packed vector of
   hk_mlp_nparams() floats, W1 (64x3), b1 (64), W2 (64x64), b2, W3 (64x64),
   b3, W4 (2x64), b4 (2), matrices row-major (outputs x inputs).  X is
   batch x 3 and Y batch x 2, row-major. */
int hk_mlp_nparams(void);
/* floats per sample of the activation cache (input + three hidden layers) */
int hk_mlp_cache_floats(void);

/* Y = net(X).  act_cache: NULL, or batch * hk_mlp_cache_floats() floats that
   receive what hk_mlp_backward needs. */
hk_status hk_mlp_forward(const float* W, const float* X, int batch, float* Y, float* act_cache,
                         hipStream_t s);

/* dW = gradient of sum(dY .* Y) over the batch with respect to W
   (overwritten, hk_mlp_nparams() floats), from the cache of the forward pass
   at the same W.  delta: scratch of batch * 192 floats.  Sums over the batch
   run in a fixed order (bitwise reproducible). */
hk_status hk_mlp_backward(const float* W, const float* act_cache, const float* dY, int batch, float* dW,
                          float* delta, hipStream_t s);

/* *loss = mean over the batch x 2 outputs of (Y - T)^2, dY = its gradient
   with respect to Y. */
hk_status hk_mlp_mse(const float* Y, const float* T, int batch, float* dY, float* loss, hipStream_t s);

/* One Adam step (Kingma & Ba 2015, Algorithm 1) at step number step >= 1:
   m, v are the moment estimates (start at zero), updated in place with W. */
hk_status hk_mlp_adam_step(float* W, float* m, float* v, const float* dW, int nparams, float lr,
                           float b1, float b2, float eps, int step, hipStream_t s);

/* ---- learned precision and shift ----------------------------------------
   Scaling of the network's inputs and outputs and the two validation
   statistics the proposal uses. */
typedef struct {
  float in_mean[3], in_scale[3];    /* features (N, beta, ln N): (x - mean) / scale   */
  float out_mean[2], out_scale[2];  /* outputs: y * scale + mean = (bits, ln lambda_1) */
  float bits_margin;                /* proposed bits = predicted bits * margin        */
  float rmse_ln_lambda;             /* validation RMSE of the predicted ln lambda_1   */
} hk_mlp_meta;

/* Proposals for count instances: bits_hat[i] = predicted bits x margin,
   rounded up to a multiple of 32 (>= 64); ln_sigma_hat[i] = predicted
   ln lambda_1 - 3 RMSE.  W: trained parameters (device); dev_io: device
   scratch of 5 * count floats.  Synchronises s. */
hk_status hk_mlp_propose(const float* W, const hk_mlp_meta* meta, const hk_instance* inst, int count,
                         float* dev_io, hipStream_t s, int* bits_hat, double* ln_sigma_hat);

/* The inertia bracket of "Interval Verification" for many instances at
   once: lambda_dec[i] (decimal scientific notation) truncated to `digits`
   significant digits, floored to K_i bits, must leave every pivot of
   M - xI positive, and one unit more in the last digit (ceiled) must give
   exactly one negative pivot, in instance i's own precision K_i =
   inst[i].prec_bits.  ok[i] = 1 when both hold.  Two batched
   factorisations; dev_ws of hk_batch_workspace_bytes(inst, count) bytes.
   Used to find the bits an instance needs.  Synchronises s. */
hk_status hk_bracket_batched(const hk_instance* inst, int count, const char* const* lambda_dec, int digits,
                             int panel, void* dev_ws, size_t ws_bytes, hipStream_t s, int* ok);

/* Device bytes hk_eig_learned needs for these instances and proposals. */
size_t hk_learned_workspace_bytes(const hk_instance* inst, int count, const int* bits_hat);

/* lambda_1 of every instance with proposed precisions and shifts (not in
   the paper).  For instance i with b = bits_hat[i] and sigma =
   exp(ln_sigma_hat[i]): M - sigma I is factored at b and at ceil(1.25 b)
   bits (all instances and both precisions in one batched factorisation;
   a pivot <= 0 halves sigma, at most three times, then sigma = 0), inverse
   iteration runs on each factorisation, and lambda(1.25 b) is accepted
   when it agrees with lambda(b) to 10^-digits relative (out[i].path = 1).
   Otherwise the precision rises by 1.25 at most twice more, each level
   compared with the one before; when nothing agrees, or the next level
   would exceed inst[i].prec_bits, the plain method runs at
   inst[i].prec_bits (inverse iteration from 0 and the inertia bracket,
   out[i].path = 0).  lambda_dec carries digits + 5 significant digits.
   rep may be NULL.  Synchronises s. */
hk_status hk_eig_learned(const hk_instance* inst, int count, const int* bits_hat, const double* ln_sigma_hat,
                         int digits, int panel, void* dev_ws, size_t ws_bytes, hipStream_t s, hk_result* out,
                         hk_batch_report* rep);

#ifdef __cplusplus
}
#endif
#endif /* HK_H */
