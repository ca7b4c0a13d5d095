/*
 * hl.h -- C ABI of libhankel: the smallest eigenvalue of the moment Hankel
 * matrix H_N = (mu_{i+j}) of the weight exp(-x^beta) on [0, inf), by an
 * extreme-precision LDL^T factorisation, the top-left k x k block of H_N^-1 and
 * the largest eigenvalue of that block (Chen, Sikorowski, Zhu, "Smallest
 * eigenvalue of large Hankel matrices at critical point", Sections 2 and 4).
 *
 * Plain C: no C++ types, no exceptions, no torch types.  Every pointer is either
 * host memory or device (HIP) memory as stated; the library never allocates
 * device memory after hl_create.  The caller owns every buffer.
 *
 * Numbers.  A "P-bit number" is nl = P/32 little-endian uint32 limbs in two's
 * complement.  A "2P-bit number" is 2*nl limbs.  The precision P must be a
 * multiple of 128 and at least 256.
 *
 * Scaled fixed point (Section 4.1, eq. precision, with the diagonal scaling of
 * Section 6.2 restricted to powers of two).  Row j carries a scale exponent s_j
 * shared by a block of E rows; the factorisation works on the integers
 * a_rc = rnd(mu_{r+c} 2^(W - s_r - s_c)), W = 2P - 4, and returns
 *   pivots       d_i  with  D_i  = d_i  2^(2 s_i - W),
 *   multipliers  b_ri with  L_ri = b_ri 2^(s_r - s_i - h_i),
 * where h_i = bitlen(d_i) / 2.  The update a_rc -= b_ri u_ci is exact; rounding
 * (to nearest, ties away from zero) happens only at the load, at the two
 * factor columns u, b of each pivot, at each entry of the first k columns of
 * L^-1, and at the final block.  Results are deterministic: the same inputs give
 * the same bits whatever the form (MFMA or VALU) or launch shape.
 *
 * Errors.  Calls are stream ordered and asynchronous unless stated.  Argument
 * errors return immediately.  Errors found on the device (a pivot that is not
 * positive, a factor that exceeds its P bits) are recorded in a status word in
 * the workspace; every later kernel of the same workspace returns at once, and
 * the status is returned by the next synchronising call (hl_sync,
 * hl_lambda_min).
 */
#ifndef HL_H
#define HL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HL_OK = 0,
  HL_EINVAL = 1,    /* bad argument (sizes, null pointers, precision)            */
  HL_ENOTPD = 2,    /* pivot d_i <= 0: precision too low or input not positive definite */
  HL_EOVERFLOW = 3, /* a P-bit quantity reached 3 * 2^(P-3): head room exhausted   */
  HL_ENOCONV = 4,   /* the eigen-step did not converge within its iteration limit */
  HL_EHIP = 5,      /* a HIP runtime call failed                                  */
  HL_ENOMEM = 6     /* a caller buffer is smaller than hl_get_sizes asks for      */
} hl_status;

enum { HL_FORM_MFMA8 = 0, HL_FORM_VALU = 1 };

typedef struct hl_ctx hl_ctx;

/* Problem shape. */
typedef struct {
  int32_t N;         /* order of H_N, 1 <= N <= 8192                                 */
  int32_t k;         /* size of the top-left block of H_N^-1, 1 <= k <= min(N, 32)    */
  int32_t prec_bits; /* P, multiple of 128, 256 <= P <= 65536                         */
  int32_t exp_block; /* E, rows sharing one scale exponent, >= 1                      */
  int32_t form;      /* HL_FORM_MFMA8: Schur update as exact int8 MFMA GEMMs;
                        HL_FORM_VALU: limb products on the vector ALU               */
} hl_shape;

/* Buffer sizes for a shape (all counts in elements of the stated type). */
typedef struct {
  size_t workspace_bytes; /* device workspace for hl_factor / hl_inv_block / hl_lambda_min */
  size_t d_words;         /* uint32: pivots, N x 2nl                                     */
  size_t l_words;         /* uint32: multipliers, N x NT x nl                            */
  size_t x_words;         /* uint32: first k columns of L^-1, NT x k x nl                */
  size_t blk_words;       /* uint32: block, k x k x nl                                   */
  int32_t nl;             /* limbs per P-bit number                                      */
  int32_t NT;             /* N rounded up to a multiple of 32                            */
  int32_t mu_limbs_min;   /* not used (moments may have any width w >= 1)                */
  int32_t reserved;
  size_t trail_offset;    /* byte offset and size in the workspace of the trailing
                             matrix kept between hl_factor_cols calls (2P-bit
                             entries in 32 x 32 tiles); copy it to checkpoint a
                             factorisation in progress                           */
  size_t trail_bytes;
  size_t diag_offset;     /* byte offset in the workspace of 64 int32 eigen-step
                             diagnostics: [1], [9] iterations of the two blocks,
                             [16..40), [40..64) per-iteration bracket bits*1000+limbs */
} hl_sizes;

/* Device views of the factorisation, all owned by the caller. */
typedef struct {
  uint32_t *d; /* device, N x 2nl limbs: pivot d_i at d + i*2nl                        */
  int32_t *h;  /* device, N: h_i = bitlen(d_i) / 2                                       */
  int32_t *s;  /* device, N: row scale exponents s_j                                     */
  uint32_t *l; /* device, N x NT x nl limbs: b_ri at l + (i*NT + r)*nl, two's
                  complement; entries with r <= i or r >= N are zero                    */
} hl_factor_t;

/* Result of the eigen-step (host). */
typedef struct {
  double lambda1;     /* 1 / lambda_max(k x k block of H^-1), rounded to double          */
  double lambda1_km1; /* the same from the leading (k-1) x (k-1) block (k >= 2)          */
  double trunc;       /* lambda1 - lambda1_km1 (<= 0), the truncation-error estimate     */
  int64_t exp;        /* lambda1 = lam_mant * 2^exp (lam_mant: nl limbs, unsigned)       */
  int64_t exp_km1;    /* lambda1_km1 = lam_mant_km1 * 2^exp_km1                          */
  int32_t iterations; /* eigen-step iterations used (both blocks)                        */
  int32_t reserved;
} hl_lambda_t;

/* One further eigenvalue from hl_lambda_next (host). */
typedef struct {
  double lambda;      /* lambda_j ~= 1 / (j-th largest eigenvalue of the k x k block)    */
  double lambda_km1;  /* the same from the leading (k-1) x (k-1) block                   */
  double trunc;       /* lambda - lambda_km1 (<= 0 by interlacing), truncation estimate  */
  int64_t exp;        /* lambda = mant * 2^exp (mant: nl limbs, unsigned)                */
  int64_t exp_km1;    /* lambda_km1 = mant_km1 * 2^exp_km1                               */
  int32_t j;          /* 2, 3                                                             */
  int32_t iterations; /* eigen-step iterations used (both blocks)                        */
} hl_lambda_j_t;

/* Context: selects the device and holds timers.  Not thread safe. */
hl_status hl_create(hl_ctx **ctx, int device);
hl_status hl_destroy(hl_ctx *ctx);

/* Human-readable detail of the last non-OK status of this thread. */
const char *hl_last_error(void);

/* Sizes of every buffer for a shape; EINVAL if the shape is not supported. */
hl_status hl_get_sizes(const hl_shape *sh, hl_sizes *out);

/*
 * hl_factor -- Algorithm 1 (serial LDL^T, no pivoting, Section 4.3) of the
 * scaled Hankel matrix, blocked in panels of 16 columns.
 *   mu      device, (2N-1) x w uint32 limbs: mantissa M_m of moment m (unsigned)
 *   mu_exp  device, 2N-1 int64: mu_m = M_m * 2^mu_exp[m]; every M_m must be > 0
 *   ws      device workspace of at least hl_sizes.workspace_bytes; it carries the
 *           status word and must be passed unchanged to hl_inv_block and
 *           hl_lambda_min of the same factorisation
 *   out     device views, sized by hl_get_sizes
 *   stream  hipStream_t (NULL: the null stream)
 * Device errors: HL_ENOTPD (index = pivot), HL_EOVERFLOW (index = column).
 */
hl_status hl_factor(hl_ctx *ctx, const hl_shape *sh, const uint32_t *mu, const int64_t *mu_exp,
                    int32_t w, void *ws, size_t ws_bytes, const hl_factor_t *out, void *stream);

/*
 * hl_factor_cols -- the same for pivots [col_begin, col_end) only: col_begin = 0
 * also loads H; later calls continue from the trailing matrix kept in ws.  Both
 * ends must be multiples of 16 (col_end may be N).  hl_factor(...) is
 * hl_factor_cols(..., 0, N, ...).  Used to time or check part of a
 * factorisation and to run one in pieces.
 */
hl_status hl_factor_cols(hl_ctx *ctx, const hl_shape *sh, const uint32_t *mu, const int64_t *mu_exp,
                         int32_t w, void *ws, size_t ws_bytes, const hl_factor_t *out,
                         int32_t col_begin, int32_t col_end, void *stream);

/*
 * hl_set_karatsuba -- form of the exact Schur update of hl_factor for
 * HL_FORM_MFMA8 shapes.  The update of Algorithm 1's inner loops is exact, so
 * every form gives the same bits; they differ in speed only.
 *   mode  0: one int8 digit-product GEMM of the P-bit factors (S = P/8 digits);
 *         1: one Karatsuba level: the factors, as S' digits (S rounded up to a
 *            multiple of 256, zero digits on top), split at digit S'/2, three
 *            GEMMs of (S'/2 + 1)-digit operands (3/4 of the int8 multiply-adds
 *            when S' = S), their exact sums combined per entry with exact
 *            carries;
 *         2: two levels: nine GEMMs of (S'/4 + 2)-digit operands (9/16);
 *         3: three levels: 27 GEMMs of (S'/8 + 3)-digit operands (27/64);
 *         4: four levels: 81 GEMMs of (S'/16 + 4)-digit operands (81/256);
 *        -1 (default): 4 from P = 40960 on, 3 from 32768, 2 from 16384, 1 from
 *            8192, else 0.
 * A mode beyond what the shape allows runs the deepest allowed one (levels
 * deeper than the default are allowed only while their products fit 16 GiB of
 * workspace).  Applies to later
 * hl_factor / hl_factor_cols calls on this context (modes may be mixed within
 * one factorisation).  HL_EINVAL for another mode.
 */
hl_status hl_set_karatsuba(hl_ctx *ctx, int32_t mode);

/*
 * hl_inv_block -- first k columns of L^-1 (Algorithm 4, Section 4.4) and the
 * top-left k x k block of H^-1 (eq. equ:index, Section 4.5).
 *   x        device, NT x k x nl limbs: x_rm at x + (r*k + m)*nl, the scaled
 *            entries of L^-1 (x_mm = 2^(Q - h_m), Q = W - G, G = max_{m<k} s_m + 64)
 *   blk      device, k x k x nl limbs: (H^-1)_ab ~= blk_ab * 2^blk_exp, |blk_ab| <= 2^(P-2)
 *   blk_exp  device, 1 int64
 * Uses the workspace's trailing-matrix region as scratch (the factorisation
 * must be complete) and, in the MFMA form, the context's second stream for
 * half of the block sums; the caller's stream waits for it, so the call stays
 * ordered on that stream.
 * Device errors: HL_EOVERFLOW (index = row of L^-1).
 */
hl_status hl_inv_block(hl_ctx *ctx, const hl_shape *sh, const hl_factor_t *f, void *ws,
                       size_t ws_bytes, uint32_t *x, uint32_t *blk, int64_t *blk_exp, void *stream);

/*
 * hl_lambda_min -- lambda_1 ~= 1 / lambda_max(block), and the same from the
 * leading (k-1) x (k-1) block for the truncation estimate (Sections 4.2 and 4.5),
 * by shifted inverse iteration with Rayleigh quotients in multiprecision
 * floating point, every shift certified by the signs of an LDL^T.  Synchronises
 * the stream; returns the first device error of the workspace if there is one.
 *   lam_mant, lam_mant_km1  optional device outputs, nl limbs each (NULL: skip)
 *   out                     host
 */
hl_status hl_lambda_min(hl_ctx *ctx, const hl_shape *sh, const uint32_t *blk, const int64_t *blk_exp,
                        void *ws, size_t ws_bytes, uint32_t *lam_mant, uint32_t *lam_mant_km1,
                        hl_lambda_t *out, void *stream);

/*
 * hl_lambda_min_noalloc -- hl_lambda_min for callers that cannot allocate
 * device memory or pass a workspace (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same results, bit for bit, from the block alone.  Its scratch (status word
 * and the eigen-step's work area) is a static device array of 64 MiB per GPU,
 * held from library load until the process ends.  That covers every precision
 * for k <= 16, P <= 36224 bits for k = 24 and P <= 20608 bits for k = 32;
 * larger shapes return HL_EINVAL.  Both blocks run on the caller's stream one
 * after the other.  Calls that overlap on one GPU share that array and race:
 * serialise them.  Every call clears the array first.  Synchronises the stream;
 * returns HL_ENOCONV (index 0 or 1, the block) if the eigen-step does not
 * converge.  Allocates no device memory.
 *   blk, blk_exp            device, as written by hl_inv_block
 *   lam_mant, lam_mant_km1  optional device outputs, nl limbs each (NULL: skip)
 *   out                     host
 */
hl_status hl_lambda_min_noalloc(hl_ctx *ctx, const hl_shape *sh, const uint32_t *blk, const int64_t *blk_exp,
                                uint32_t *lam_mant, uint32_t *lam_mant_km1, hl_lambda_t *out, void *stream);

/*
 * hl_lambda_next -- lambda_2 and lambda_3 with their truncation estimates (the
 * further columns of Table 2; the estimate as in Section 4.5): the j-th
 * smallest eigenvalue of H_N taken as 1 / (j-th largest eigenvalue of the
 * block), for the k x k block and its leading (k-1) x (k-1) block.  Each
 * eigenvalue comes from the block deflated by the eigenpairs found before it,
 * B - mu y y^T / (y^T y) in the eigen-step's multiprecision floating point, and
 * the same certified inverse iteration as hl_lambda_min.  Needs hl_lambda_min
 * on the same workspace first (it uses that call's eigenvectors).  Synchronises
 * the stream; returns the first device error of the workspace if there is one.
 *   count            1 (lambda_2) or 2 (lambda_2, lambda_3); EINVAL unless k >= count + 2
 *   mant, mant_km1   optional device outputs, count x nl limbs each (NULL: skip)
 *   out              host, count entries (out[j - 2] for lambda_j)
 * Device errors: HL_ENOCONV (index = 2 (j - 1) for the k x k block, + 1 for the other).
 */
hl_status hl_lambda_next(hl_ctx *ctx, const hl_shape *sh, const uint32_t *blk, const int64_t *blk_exp,
                         void *ws, size_t ws_bytes, int32_t count, uint32_t *mant, uint32_t *mant_km1,
                         hl_lambda_j_t *out, void *stream);

/*
 * hl_lambda_grad -- the derivative of lambda_1 along a moment direction dmu
 * (dmu = d mu / d beta gives d lambda_1 / d beta).  The paper computes lambda_1
 * (Sections 4.2 and 4.5) but does not differentiate it; this is the first-order
 * perturbation of the block's largest eigenvalue:
 *   d lambda_1 = v^T dH v,  v = lambda_1 H^-1 E y  (y the unit eigenvector of
 *   the block for lambda_max, E the first k columns of I, dH_ij = dmu_{i+j}),
 * i.e. sum_m mubar_m dmu_m with the moment adjoint mubar_m = sum_{i+j=m} v_i v_j.
 * It runs on the scaled factor: one transposed triangular solve with B^T
 * (B_ri = b_ri, B_ii = 2^h_i) and an exact contraction with the scaled matrix
 * dmu_{i+j} 2^(W' - s_i - s_j); nothing but the final number is floating point.
 * Needs hl_factor, hl_inv_block and hl_lambda_min on the same workspace first.
 * Synchronises the stream.
 *   x        device, the first k columns of L^-1 written by hl_inv_block
 *   blk_exp  device, the block exponent written by hl_inv_block
 *   dmu      device, (2N-1) x w uint32 limbs: |dmu_m| (unsigned mantissa)
 *   dmu_exp  device, 2N-1 int64: |dmu_m| = mantissa * 2^dmu_exp[m]
 *   dmu_neg  device, 2N-1 int32: nonzero where dmu_m < 0
 *   z        optional device output, N x nl limbs (two's complement): the
 *            adjoint vector in the scaled basis, v_i = lambda_1 2^(W - s_i - F)
 *            z_i / ynorm with F = out->z_shift (NULL: not written)
 *   out      host; besides the double result it locates the exact integers
 *            the result is made of, in the workspace until its next use:
 *            dlambda1 = lambda_1^2 * num * 2^num_shift / den, num two's
 *            complement (num_limbs limbs at byte offset num_offset), den > 0
 *            (den_limbs limbs at den_offset)
 * Device errors: HL_EOVERFLOW (index = row of z) when z leaves its P bits.
 */
typedef struct {
  double dlambda1;     /* sum_m (d lambda_1 / d mu_m) dmu_m                          */
  double lambda1;      /* lambda_1 of the same factorisation                         */
  double ynorm;        /* |y| of the eigenvector used (its largest entry in [1/2, 1)) */
  int64_t z_shift;     /* F, the binary point of z                                   */
  int64_t num_shift;
  uint64_t num_offset;
  uint64_t den_offset;
  int32_t num_limbs;
  int32_t den_limbs;
} hl_grad_t;
hl_status hl_lambda_grad(hl_ctx *ctx, const hl_shape *sh, const hl_factor_t *f, const uint32_t *x,
                         const int64_t *blk_exp, const uint32_t *dmu, const int64_t *dmu_exp,
                         const int32_t *dmu_neg, int32_t w, void *ws, size_t ws_bytes, uint32_t *z,
                         hl_grad_t *out, void *stream);

/*
 * Batches (many instances of uneven N and precision in one launch sequence).
 * The paper factors one matrix at a time on a cluster and hands the largest
 * work out first (Section 4.3.3); here a batch advances all its instances in
 * lock step over a global pivot counter, every launch covering every instance
 * that still has work (so the sequential chain of Algorithm 1 is paid once per
 * batch), the trailing updates of a step go to one persistent int8 MFMA launch
 * fed from per-XCD queues of work items, largest first (an instance in the
 * Karatsuba form contributes its 3^L digit-sum products, combined into its
 * trailing matrix after the launch), and the whole sequence
 * (load, panels, the first k columns of L^-1, the blocks, the eigen-steps) is
 * captured once in a hipGraph and replayed.  Results are bit-identical to
 * hl_factor + hl_inv_block + hl_lambda_min on each instance.
 */
typedef struct {
  hl_shape shape;          /* as for hl_factor (form may be overridden by the tuning) */
  const uint32_t *mu;      /* device moments, (2N-1) x w limbs                        */
  const int64_t *mu_exp;   /* device, 2N-1                                            */
  int32_t w;
  void *ws;                /* device workspace of hl_get_sizes(shape) bytes           */
  size_t ws_bytes;
  hl_factor_t f;           /* device outputs as for hl_factor                         */
  uint32_t *x;             /* device outputs as for hl_inv_block                      */
  uint32_t *blk;
  int64_t *blk_exp;
} hl_instance;

/* Launch shape of a batch (never changes the results). */
typedef struct {
  int32_t items_per_simd;  /* MFMA work items per SIMD and step (granularity)        */
  int32_t range_cap;       /* most output-limb ranges per tile                        */
  int32_t valu_below_bits; /* instances with P below this use the VALU update form   */
  int32_t karatsuba;       /* trailing-update form of MFMA-form instances: 0 by
                              precision (as hl_set_karatsuba(-1)), -1 the digit
                              product, 1 .. 3 that many Karatsuba levels          */
} hl_tune_t;

typedef struct hl_batch hl_batch;

/* Bytes of device memory the batch's launch plan needs (argument tables and
 * work queues); tune may be NULL (defaults). */
hl_status hl_batch_plan_bytes(int32_t count, const hl_instance *inst, const hl_tune_t *tune, size_t *bytes);

/* Build the plan into the caller's device buffer `plan` (which must stay
 * allocated and untouched while the batch exists) and capture the whole launch
 * sequence in a hipGraph.  Instances must not share workspaces or outputs. */
hl_status hl_batch_create(hl_ctx *ctx, int32_t count, const hl_instance *inst, const hl_tune_t *tune,
                          void *plan, size_t plan_bytes, hl_batch **out);
/* Replay the graph on `stream` (asynchronous). */
hl_status hl_batch_launch(hl_batch *b, void *stream);
/* Wait for `stream`; per-instance lambda_1 results (host arrays of count) and
 * device status (HL_OK or the instance's first device error). */
hl_status hl_batch_results(hl_batch *b, void *stream, hl_lambda_t *out, hl_status *status);
hl_status hl_batch_destroy(hl_batch *b);

/* Autotuner: builds and times the batch's first `panels` panel steps under each
 * candidate launch shape (items per SIMD 2, 4, 8; range cap 16, 64; VALU
 * below 0, 4096 bits; Karatsuba by precision or the digit product) and returns
 * the fastest in *best (its time per replay in *best_ms).  Uses the instances'
 * workspaces and `plan` as scratch. */
hl_status hl_autotune(hl_ctx *ctx, int32_t count, const hl_instance *inst, void *plan, size_t plan_bytes,
                      int32_t panels, hl_tune_t *best, double *best_ms);

/* Wait for the stream and return the status word of the workspace (index of
 * the failing pivot or column in *index if not NULL). */
hl_status hl_sync(hl_ctx *ctx, void *ws, void *stream, int32_t *index);

/* Per-stage device time of the last hl_factor / hl_inv_block / hl_lambda_min on
 * this context, measured with HIP events on the caller's stream when timing is
 * enabled (hl_set_timing(ctx, 1); timing synchronises after each stage).
 * ms[0] Schur update (all its kernels), ms[1] panel (pivots, factor columns,
 * in-panel updates), ms[2] triangular solve, ms[3] block, ms[4] eigen-step,
 * ms[5] load, ms[6] the int8 MFMA GEMM kernel alone, ms[7] whole hl_factor,
 * ms[8] hl_lambda_grad, ms[9] the Karatsuba combination kernel alone;
 * launches[0] Schur updates, launches[1] MFMA GEMM launches, launches[2] those
 * of them in a Karatsuba form, launches[3] the sum of their levels. */
typedef struct {
  double ms[12];
  int64_t launches[4];
  double schur_limb_macs; /* algorithmic limb multiply-adds of the Schur updates */
} hl_timing_t;
hl_status hl_set_timing(hl_ctx *ctx, int enable);
hl_status hl_get_timing(hl_ctx *ctx, hl_timing_t *out);

/* Iteration limit of the eigen-step of hl_lambda_min and hl_lambda_min_noalloc
 * on this context, per block: 0 (the default) keeps the built-in limit of 400;
 * a smaller limit makes a call that needs more iterations return HL_ENOCONV
 * with the block as index (0: the k x k block, 1: the leading (k-1) x (k-1)
 * block).  For exercising that error path; EINVAL for a negative limit. */
hl_status hl_set_eig_maxit(hl_ctx *ctx, int32_t maxit);

/* Test hooks (not part of the method): exact products and the pivot
 * reciprocal on the device, for checking the multi-limb primitives against
 * host integers. */
hl_status hl_debug_mul(const uint32_t *a, int32_t na, const uint32_t *b, int32_t nb, uint32_t *out,
                       int32_t nout, void *stream);
hl_status hl_debug_recip(const uint32_t *d, int32_t nd, int32_t P, uint32_t *omega, int32_t *h,
                         void *stream);
/* Issue-rate probe of the vector ALU's 32 x 32 -> 64-bit integer multiply-add,
 * the limb product of the HL_FORM_VALU Schur update: `blocks` workgroups of 256
 * threads, each thread running 8 independent chains of `iters` steps (mode 0:
 * v_mad_u64_u32 plus v_addc_co_u32 of its carry, the form's pair; mode 1:
 * v_mad_u64_u32 alone), operands in registers: blocks * 256 * iters * 8
 * multiply-adds.  sink: device, one uint64 (written only on an impossible
 * value).  Time it with events on `stream`. */
hl_status hl_debug_valu_peak(int32_t mode, int32_t blocks, int32_t iters, uint64_t *sink, void *stream);
/* out[0..nout) = a b mod 2^(32 nout) for non-negative a (na limbs) and b (nb
 * limbs), all device pointers, by the one-workgroup int8 MFMA product that the
 * pivot reciprocal uses (threads: 256 or 1024 per workgroup).  HL_EHIP when the
 * operands and scratch exceed the 160 KiB of LDS. */
hl_status hl_debug_mul_wg(const uint32_t *a, int32_t na, const uint32_t *b, int32_t nb, uint32_t *out,
                          int32_t nout, int32_t threads, void *stream);
/* Output layout of v_mfma_i32_32x32x32_i8: out (device, 2048 int32) holds, per
 * accumulator register v and lane l at out[v*64 + l], 32(m+1) for A rows m+1,
 * B ones, then at out[1024 + v*64 + l] 32(n+1) for A ones, B columns n+1. */
hl_status hl_debug_mfma_layout(int32_t *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HL_H */
