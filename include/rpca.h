/*
 * rpca.h -- C ABI of the MI355X (gfx950) DCF-PCA library.
 *
 * DCF-PCA (arXiv 2207.11669, Algorithm 1 in Section 2.2) minimises
 *
 *     1/2 ||U V^T + S - M||_F^2 + rho/2 (||U||_F^2 + ||V||_F^2) + lambda ||S||_1
 *
 * (Section 1, the nonconvex factorised objective) with M = [M_1 ... M_E] split
 * column-wise over E clients (Section 2.1). Every round broadcasts U, lets each
 * client take K local steps -- the (V_i, S_i) argmin of eq. "VS_arg" followed by
 * a U step (eq. "U_local") -- and replaces U by the mean of the client factors
 * (eq. "U_agg"). All clients live on one GPU; the mean is a device reduction.
 *
 * Conventions shared by every entry point:
 *  - All matrices are column-major FP32 in device memory unless stated.
 *  - Status codes: RPCA_OK (0) on success, negative on error, positive for a
 *    warning on an otherwise successful call. rpca_last_error() gives text.
 *  - A context is bound to one HIP stream; every call enqueues on that stream
 *    and is asynchronous unless it says it synchronises. A context is not
 *    thread-safe.
 *  - Device errors poison the context: later calls return RPCA_ESTATE.
 */
#ifndef RPCA_H_
#define RPCA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpca_ctx rpca_ctx;

typedef enum {
  RPCA_OK = 0,
  RPCA_EINVAL = -1,      /* bad argument; nothing was enqueued */
  RPCA_EWORKSPACE = -2,  /* workspace missing, too small or misaligned */
  RPCA_EDEVICE = -3,     /* a HIP call failed; the context is poisoned */
  RPCA_ENONFINITE = -4,  /* a non-finite objective was observed; poisoned */
  RPCA_ESTATE = -5,      /* the context is poisoned or not initialised */
  RPCA_WARN_THM2 = 1     /* rho^2 > lambda^2 m n: by Theorem 2 (Section 3.3) the
                            iterates can only reach U = 0 */
} rpca_status;

/* U step taken by each client after its (V_i, S_i) update. */
typedef enum {
  RPCA_U_GRAD = 0,   /* U_i <- U_i - eta grad_U L_i (eq. "U_local", Lemma 2) */
  RPCA_U_CLOSED = 1  /* U_i <- argmin_U L_i(U, V_i, S_i)
                        = (M_i - S_i) V_i (V_i^T V_i + rho n_i/n I)^{-1} */
} rpca_u_mode;

/* Step-size schedule for RPCA_U_GRAD (indexed by round t = 0, 1, ...). */
typedef enum {
  RPCA_ETA_CONST = 0,  /* eta_t = eta0 */
  RPCA_ETA_SQRT = 1    /* eta_t = eta0 / sqrt(t + 1): a decaying rate (Section 4.2) */
} rpca_eta_sched;

/* Size limits (rpca_params_error names the one a problem breaks). Besides the
 * per-field ranges below, the kernels address whole factor layouts with 32-bit
 * byte ranges, so with RP = r rounded up to 16:
 *   (m rounded up to 128) * RP * 4 < 2^31          (m < 2^23 at r = 64), and
 *   (sum of the n_i each rounded up to 64) * RP * 4 < 2^31
 *                                                   (n < 2^23 at r = 64).
 * Ranks above 64 (the upper-bound rank experiments of Section 4.2 and Table 1
 * fit up to 0.2 n) run in FP32 only: RPCA_FLAG_BF16 and RPCA_FLAG_BF16X3
 * need r <= 64, and the launch shape keeps one column group per V-pass wave
 * and one S-pass column phase. A client narrower than r makes V_i^T V_i
 * singular; the closed-form U step then amplifies the FP32 rounding of
 * (M_i - S_i) V_i by up to n / (rho n_i). */
typedef struct {
  int64_t m;               /* rows of M (all clients share them), 1 <= m < 2^26 */
  int32_t E;               /* number of clients, 1 <= E <= 4096 */
  const int64_t* n_cols;   /* host array [E]: 1 <= n_i <= 2^30 columns of client i */
  int32_t r;               /* factor rank, 1 <= r <= 128 */
  double rho;              /* rho > 0 (Frobenius penalty on U and V) */
  double lambda;           /* lambda >= 0 (l1 penalty on S) */
  int32_t K;               /* local steps per round, K >= 1 (Algorithm 1) */
  int32_t inner;           /* (V, S) alternations per local step, >= 1 */
  int32_t u_mode;          /* rpca_u_mode */
  double eta0;             /* step size for RPCA_U_GRAD (> 0 there) */
  int32_t eta_sched;       /* rpca_eta_sched */
  uint32_t flags;          /* RPCA_FLAG_* bits */
  uint64_t seed;           /* seed of the U^(0) draw when rpca_init gets U0 = NULL */
} rpca_params;

/* With K = 1 and one alternation the library does not store S between rounds:
 * the V-pass rebuilds S_i^(t) = soft(M_i - U^(t-1) V_i^(t)T) (eq. "optS") from
 * the previous round's factors, which halves the HBM traffic of a round. This
 * flag keeps S in the workspace instead (the layout used for K > 1 or more
 * than one alternation); the results agree to FP32 rounding. */
#define RPCA_FLAG_STORE_S 1u
/* Replay steady-state rounds from HIP graphs: rpca_step captures two
 * consecutive rounds (K = 1, one alternation, S rebuilt) once per buffer
 * parity and launches the graph for every later pair of rounds, which removes
 * the host cost of the per-round launches. Results are bitwise those of the
 * eager launches. Needs a stream other than the null stream (rpca_init
 * returns RPCA_EINVAL otherwise); ignored with RPCA_FLAG_STORE_S, K > 1 or
 * inner > 1. */
#define RPCA_FLAG_GRAPH 2u
/* Mixed precision. rpca_init makes two BF16 copies of M (2 B per entry each,
 * in the operand layouts of the two streaming passes) and the factor kernels
 * keep BF16 copies of U and V next to the FP32 ones. While the context's
 * precision is RPCA_PREC_BF16 (the initial precision with this flag), the
 * rank-r contractions of a round take M, U and V in BF16 with FP32
 * accumulation, so each streaming pass reads 2 B per entry of M instead of 4.
 * The residual, soft-threshold, Lambda, the U step and all statistics stay
 * FP32/FP64, and the factors are FP32 throughout. rpca_set_precision switches
 * to FP32 rounds (which read the caller's FP32 M) at any round boundary: the
 * FP32 closing rounds refine the BF16 iterate to the FP32 fixed point.
 * Needs K = 1, inner = 1 and no RPCA_FLAG_STORE_S. rpca_get_LS evaluates S in
 * FP32 from the current factors in either precision.
 * Applicability: BF16 keeps 8 significand bits, so an entry x of M, U V^T or
 * Lambda is off by up to 2^-9 |x|. The soft-threshold resolves the residual
 * only to lambda, so BF16 rounds follow the FP32 iteration only while lambda
 * is well above 2^-9 times the typical size of the low-rank part's entries;
 * below that their Lambda is rounding noise and the iterates stall far from
 * the FP32 fixed point. */
#define RPCA_FLAG_BF16 4u
/* Three-product BF16 rounds (RPCA_PREC_BF16X3) without the BF16 copies of M:
 * the factor kernels keep BF16 hi/lo splits of U and V (hi = BF16(x),
 * lo = BF16(x - hi), 16 significand bits together), and each rank-r product
 * runs as three BF16 MFMA products (hi.hi + hi.lo + lo.hi) with FP32
 * accumulation, reading M in FP32 from the caller's blocks (4 B per entry,
 * as FP32 rounds). The products are then accurate to about 2^-17 relative,
 * far below lambda on every workload here, at a third of FP32 MFMA's work
 * per product on the BF16 units. Needs K = 1, inner = 1, no
 * RPCA_FLAG_STORE_S and every ldm < 2^24. RPCA_FLAG_BF16 also keeps the
 * splits, so a context with it can run either BF16 precision. */
#define RPCA_FLAG_BF16X3 8u
/* Sparse S between the passes of FP32 rounds. Each FP32 S-pass also writes
 * the S it forms (eq. "optS") in sparse form: per 16 x 16 tile of (row,
 * padded column), four 64-bit support words and the nonzero values packed in
 * order. The next round's V-pass reads that instead of rebuilding S from the
 * previous factors: about 0.125 B per entry plus 4 B per nonzero of extra
 * traffic, 2 r fewer flops per entry. S is the same bit for bit, so results
 * are bitwise those without the flag. A round rebuilds S as without the flag
 * when the previous round was not an FP32 round or ran at another lambda.
 * Workspace: (n rounded per client to 64) x (m rounded to 128) x 4.125 bytes
 * more. Needs K = 1, inner = 1 and no RPCA_FLAG_STORE_S. */
#define RPCA_FLAG_SPARSE_S 16u

/* Arithmetic of a round's streaming passes (rpca_set_precision). */
typedef enum {
  RPCA_PREC_FP32 = 0,
  RPCA_PREC_BF16 = 1,   /* needs a context created with RPCA_FLAG_BF16 */
  RPCA_PREC_BF16X3 = 2  /* needs RPCA_FLAG_BF16X3 or RPCA_FLAG_BF16 */
} rpca_precision;

/* Per-round statistics, FP64, recorded at the last local step of round t:
 * objective = sum_i L_i(U_i, V_i, S_i) with U_i the client factor that the
 * (V_i, S_i) update used (Section 2.2 local objectives; for K = 1 this is the
 * global objective at (U^(t), V^(t+1), S^(t+1))), at the round's lambda;
 * lambda_fro_sq = ||M - U V^T - S||_F^2; nnz = number of nonzeros of S;
 * du_sq = ||U^(t+1) - U^(t)||_F^2; u_sq = ||U^(t+1)||_F^2; v_sq = ||V||_F^2;
 * l1 = ||S||_1; objective_target = the same objective at the problem's own
 * lambda with S at its optimum for the round's factors, sum of H_lambda(M -
 * U V^T) + the penalties (Appendix A.2's Huber identity; equal to objective
 * in rounds at that lambda). A lambda schedule's rounds can be judged by it. */
typedef struct {
  double t, objective, lambda_fro_sq, nnz, du_sq, u_sq, v_sq, l1, objective_target;
} rpca_stats;

/* NULL when the parameters are valid, else a static text naming the first
 * violated condition (the checks rpca_init and rpca_workspace_bytes apply). */
const char* rpca_params_error(const rpca_params* p);

/* Bytes of device workspace rpca_init needs for these parameters.
 * Returns RPCA_EINVAL for invalid parameters (same checks as rpca_init). */
rpca_status rpca_workspace_bytes(const rpca_params* p, size_t* bytes);

/* Create a context (Algorithm 1, initialisation step).
 *  M_blocks: host array [E] of device pointers; M_blocks[i] is client i's
 *            m x n_i block, column-major with leading dimension ldm[i].
 *            Borrowed, read-only, and must stay valid while the context
 *            lives. Each pointer must be 16-byte aligned, m <= ldm[i] < 2^26
 *            and ldm[i] % 4 == 0.
 *  U0:       device m x r column-major start U^(0) with leading dimension
 *            ldu >= m (copied; not retained), or NULL: Algorithm 1 leaves the
 *            start open, and the library then draws U^(0) on the device with
 *            i.i.d. N(0, 1) entries from p->seed. Entry (i, c) uses the
 *            outputs j = 2k and 2k + 1, k = c m + i, of the counter form of
 *            SplitMix64 (Steele, Lea and Flood, 2014): x_j = mix(seed +
 *            (j + 1) 0x9E3779B97F4A7C15 mod 2^64), mix(z) = z ^= z >> 30,
 *            z *= 0xBF58476D1CE4E5B9, z ^= z >> 27, z *= 0x94D049BB133111EB,
 *            z ^= z >> 31; u_j = (x_j >> 11) 2^-53; and the Box-Muller value
 *            sqrt(-2 ln(1 - u_2k)) cos(2 pi u_2k+1), formed in FP64 and
 *            rounded to FP32.
 *  workspace/ws_bytes: caller-owned device memory of at least
 *            rpca_workspace_bytes() bytes, 256-byte aligned; the library
 *            allocates no device memory of its own.
 *  stream:   hipStream_t (as void*) all work is enqueued on; NULL = default.
 * S_i^(0) = 0. Returns RPCA_WARN_THM2 (context still valid) when
 * rho^2 > lambda^2 m n. On error *out is NULL and rpca_last_error(NULL)
 * names the cause. */
rpca_status rpca_init(rpca_ctx** out, const rpca_params* p,
                      const float* const* M_blocks, const int64_t* ldm,
                      const float* U0, int64_t ldu,
                      void* workspace, size_t ws_bytes, void* stream);

/* rpca_init for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * workspace is a static device array of the library,
 * RPCA_STATIC_WORKSPACE_BYTES per GPU, which each GPU the library runs on
 * holds until the process ends. The call allocates no device memory and
 * calls no allocating routine; inputs, parameters, stream and every later
 * call behave as with rpca_init. The GPU is the current device.
 *  - Parameters whose rpca_workspace_bytes exceed the array are refused with
 *    RPCA_EWORKSPACE (rpca_last_error(NULL) gives both sizes).
 *  - The array is shared by every context created this way on one GPU, so at
 *    most one such context may live per GPU: a second rpca_init_static there
 *    returns RPCA_ESTATE until the first is destroyed. The array keeps the
 *    last context's contents; rpca_init_static clears it as rpca_init clears
 *    its workspace. Calls from several threads that overlap on one GPU race.
 */
#define RPCA_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
rpca_status rpca_init_static(rpca_ctx** out, const rpca_params* p,
                             const float* const* M_blocks, const int64_t* ldm,
                             const float* U0, int64_t ldu, void* stream);

/* Enqueue `rounds` rounds of Algorithm 1 (rounds >= 0). Asynchronous. */
rpca_status rpca_step(rpca_ctx* c, int32_t rounds);

/* Run rounds until the stopping metric is <= tol or max_rounds rounds are
 * done, checking every check_every rounds (synchronises at each check).
 * The metric is ||L^(t) - L_ref||_F / ||L_ref||_F computed from factor Gram
 * matrices: L_ref is the planted target when rpca_set_target was called,
 * else the L of the previous check (relative change). *rounds_done and
 * *metric (both optional) receive the rounds run by this call and the last
 * metric. Returns RPCA_ENONFINITE if the objective became non-finite. */
rpca_status rpca_solve(rpca_ctx* c, int32_t max_rounds, double tol, int32_t check_every,
                       int32_t* rounds_done, double* metric);

/* Register a planted low-rank target L* = Ustar Vstar^T for the solve metric
 * (Section 4.1 evaluation). Ustar: device m x rstar column-major (ld ldus);
 * Vstar: device n x rstar column-major (ld ldvs), rows ordered as the
 * clients' columns. Copied into the workspace. 1 <= rstar <= 128. */
rpca_status rpca_set_target(rpca_ctx* c, const float* Ustar, int64_t ldus,
                            const float* Vstar, int64_t ldvs, int32_t rstar);

/* Relative error ||U V^T - L_ref||_F / ||L_ref||_F of the current iterate
 * against the target (or, with no target, NaN). Synchronises. */
rpca_status rpca_target_error(rpca_ctx* c, double* relerr);

/* Algorithm 1's output for client `client` (or all clients when client = -1):
 * L_i = U^(T) V_i^T and S_i, written column-major into device buffers L and S
 * with leading dimensions ldl, lds >= m (either pointer may be NULL to skip).
 * For client = -1 the buffers hold all n columns in client order. Async. */
rpca_status rpca_get_LS(rpca_ctx* c, int32_t client, float* L, int64_t ldl,
                        float* S, int64_t lds);

/* Current factors: U (m x r, ld ldu) and V (n x r, ld ldv), both column-major
 * device buffers; either may be NULL. V's rows follow the clients' columns. */
rpca_status rpca_get_factors(rpca_ctx* c, float* U, int64_t ldu, float* V, int64_t ldv);

/* Statistics of round `round` (0-based; -1 = the last finished round); only
 * the last 4096 rounds are kept. Synchronises. */
rpca_status rpca_get_stats(rpca_ctx* c, int64_t round, rpca_stats* out);

/* Kernel phases of one local step, for rpca_profile. */
typedef enum {
  RPCA_PHASE_VPASS = 0,          /* V_i ridge solve, streaming part: W = (M_i - S_i)^T U */
  RPCA_PHASE_SPASS = 1,          /* fused U V_i^T, soft-threshold into S_i, Lambda V_i */
  RPCA_PHASE_CLIENT_FACTOR = 2,  /* per-client r x r factors of the closed U step */
  RPCA_PHASE_UUPDATE = 3,        /* U step and consensus mean, Gram partials */
  RPCA_PHASE_FINALIZE = 4,       /* r x r Gram, its FP64 inverse, round statistics */
  RPCA_PHASE_VFINAL = 5,         /* V_i ridge solve, finishing part: V = W G^{-1}, V_i^T V_i */
  RPCA_NUM_PHASES = 6
} rpca_phase;

/* Measurement hook: run `rounds` rounds like rpca_step, with a HIP event pair
 * around every kernel launch, synchronise, and return per phase the average
 * launch duration in milliseconds (avg_ms[RPCA_NUM_PHASES]) and the number of
 * launches (launches[RPCA_NUM_PHASES]). The rounds count as real rounds. */
rpca_status rpca_profile(rpca_ctx* c, int32_t rounds, double* avg_ms, int64_t* launches);

/* Launch shapes of the streaming passes. None changes what a round
 * computes beyond the summation orders of W = (M_i - S_i)^T U and
 * P = Lambda V_i: results stay within FP32 rounding of one another and are
 * deterministic for a given shape. */
typedef struct rpca_launch_shape {
  /* V-pass row splits (the split-K of W over m): 1 .. twice the default
   * count, or 8 if that is more (at most one split per 64 rows); rounded so
   * that each split holds a multiple of 16 rows (32 in contexts that may run
   * BF16 rounds), so the count in effect can be lower */
  int32_t vsplit;
  /* 16-column groups per FP32 V-pass wave: 1 (waves on distinct columns share
   * U operands through the cache) or 4 (a wave takes all 64 columns of its
   * tile, the waves splitting the rows); 1 only for r > 64. In BF16 rounds
   * it picks the V-pass form: 4, the U operands in each wave's registers
   * (waves split the rows of a 64-column tile); 1, a work-group takes four
   * 64-column tiles over the same rows and copies a chunk's U operands into
   * LDS once for its four waves. Three-product rounds always run the LDS
   * form: 4, two tiles per work-group; 1, one. */
  int32_t vcols;
  /* FP32 S-pass column phases: 2 (work-groups of 8 waves, two per 32-row
   * strip taking alternate 16-column chunks, their partial P summed at the
   * end) or 1 (4 waves, one per strip); 1 only for r > 64. In BF16 rounds it
   * picks the S-pass form: 2, the V operands in each wave's registers (waves
   * of 64 rows, two column phases); 1, four waves of 32 rows over the same
   * chunks, which copy a chunk's V operands into LDS once. Three-product
   * rounds always run the LDS form. */
  int32_t sphases;
  /* Launch forms of the V-pass and the S-pass: 0, one work-group per tile
   * (a 64-column group by row split, or a 128-row block of a client); 1, a
   * persistent launch of the work-groups resident at once, each taking tiles
   * in the same order from a queue in the workspace until none is left. Each
   * tile writes its own slots of the partial sums, so both forms give
   * bitwise the same results. */
  int32_t vqueue;
  int32_t squeue;
  /* With RPCA_FLAG_SPARSE_S: 1 (the default), FP32 rounds hand S from the
   * S-pass to the next V-pass in sparse form; 0, they rebuild it as without
   * the flag (the sparse form pays where r is large and S sparse). Always 0
   * in a context without the flag. Both give bitwise the same results. */
  int32_t sparse;
} rpca_launch_shape;

/* Autotuner for the launch shapes. First the V-pass: candidates are the
 * default row-split count, half of it, two, three and four times it, and the
 * most the workspace holds (the work-group count decides how full the last
 * wave of work-groups runs), each with 1 and 4 column groups, at the current
 * S-pass shape. Then,
 * when the rounds run in FP32 or BF16, the S-pass at the chosen V-pass
 * shape: two column phases and one. Then the launch forms (per-tile grid or tile queue)
 * of the two passes, four combinations. Last, with RPCA_FLAG_SPARSE_S and
 * FP32 rounds, sparse S or rebuilt S, each with both V-pass launch forms. Each stage times its candidates in
 * turn, twice over, and compares the sums. Every timing runs `rounds` timed rounds (plus one
 * untimed); the fastest candidate is kept and returned in *out (optional).
 * Synchronises. The rounds are real rounds of the method; the choice depends
 * on timing. For r > 64 the column groups and S-pass phases stay at 1. */
rpca_status rpca_autotune(rpca_ctx* c, int32_t rounds, rpca_launch_shape* out);

/* The launch shapes in effect. */
rpca_status rpca_get_launch_shape(rpca_ctx* c, rpca_launch_shape* out);

/* Set the launch shapes (for reproducible runs); every field must be valid
 * (RPCA_EINVAL otherwise, shapes unchanged). Drops captured graphs. */
rpca_status rpca_set_launch_shape(rpca_ctx* c, const rpca_launch_shape* shape);

/* Copy the whole iterate of src into dst: factors, the S state, statistics,
 * round count, precision, lambda and launch shape (not the borrowed M or the
 * BF16 copies of it, which dst keeps). Both contexts must come from the same
 * parameters (RPCA_EINVAL otherwise); they may borrow different M buffers
 * of equal content. Synchronises src's stream, then enqueues the copy on
 * dst's. For lookahead searches: branch a trajectory, try a choice, and
 * compare. */
rpca_status rpca_copy_state(rpca_ctx* dst, rpca_ctx* src);

/* lambda of the rounds enqueued from now on (lambda >= 0, finite), for a
 * lambda schedule such as a continuation from a large value down to the
 * target. Every soft-threshold of round t uses its lambda_t, including the
 * V-pass's rebuild of S^(t) from the previous factors, and so does the
 * round's recorded objective. Needs the rebuilt-S form (K = 1, inner = 1, no
 * RPCA_FLAG_STORE_S); RPCA_EINVAL otherwise. A change drops captured graphs.
 * The paper fixes lambda; a schedule changes the path, and the method's
 * fixed point is that of the last lambda. */
rpca_status rpca_set_lambda(rpca_ctx* c, double lambda);

/* Multiplier omega of the U step for the rounds enqueued from now on:
 * U^(t+1) = U^(t) + omega (mean_i U_i - U^(t)) (eq. "U_agg" relaxed; with
 * the gradient step this is the step size omega eta, Theorem 1 asks
 * eta < 1/L). omega = 1 (the default) is the method's step, computed exactly
 * as without the multiplier. 0 < omega <= 4, else RPCA_EINVAL. A change drops
 * captured graphs. For step-size control (the library's controller). */
rpca_status rpca_set_step(rpca_ctx* c, double omega);

/* Precision of the rounds enqueued from now on (rpca_precision). BF16 needs
 * a context created with RPCA_FLAG_BF16, BF16X3 one with RPCA_FLAG_BF16X3 or
 * RPCA_FLAG_BF16 (RPCA_EINVAL otherwise). Switching drops captured graphs.
 * The next round's V-pass rebuilds S^(t) from the previous factors in the
 * new precision. A context created with RPCA_FLAG_BF16X3 only starts in
 * BF16X3. */
rpca_status rpca_set_precision(rpca_ctx* c, int32_t precision);

/* A small MLP for round-by-round control (a learned lambda schedule and U
 * step): RPCA_MLP_IN = 10 inputs, two tanh layers of RPCA_MLP_HIDDEN = 64
 * units, and RPCA_MLP_OUT = 2 outputs y_k = lo_k + (hi_k - lo_k) sigmoid(z_k):
 * y_0 in [RPCA_MLP_GMIN, 1], a per-round decay of the lambda scale, and y_1 in
 * [RPCA_MLP_WMIN, RPCA_MLP_WMAX], a multiplier of the U step (rpca_set_step).
 * Parameters are one FP32 device array of rpca_mlp_param_count() floats, in
 * this order: W1 (64 x 10, row-major), b1 (64), W2 (64 x 64), b2 (64), W3
 * (2 x 64), b3 (2). Not part of Algorithm 1; the library's own controller
 * runs on it. */
#define RPCA_MLP_IN 10
#define RPCA_MLP_HIDDEN 64
#define RPCA_MLP_OUT 2
#define RPCA_MLP_GMIN 0.5f
#define RPCA_MLP_WMIN 0.5f
#define RPCA_MLP_WMAX 2.0f
int64_t rpca_mlp_param_count(void);

/* y[i] = MLP(x[i]) for n samples (x: n x 10 row-major, y: n x 2 row-major;
 * device pointers). Enqueued on `stream` (hipStream_t as void*, NULL =
 * default). */
rpca_status rpca_mlp_forward(const float* params, const float* x, int64_t n, float* y,
                             void* stream);

/* One step of gradient descent on the mean over n samples of
 * 1/2 ||MLP(x[i]) - target[i]||^2 (target: n x 2 row-major): params -= lr *
 * mean gradient, the samples' gradients summed in index order (bitwise
 * reproducible). grad_ws: device scratch of n * rpca_mlp_param_count()
 * floats. 1 <= n <= 65535. */
rpca_status rpca_mlp_train_step(float* params, const float* x, const float* target, int64_t n,
                                float lr, float* grad_ws, void* stream);

/* Rounds enqueued so far. */
int64_t rpca_rounds(const rpca_ctx* c);

/* Text of the last error on this context (never NULL). With c = NULL: the
 * cause of the last failed context creation on the calling thread (empty if
 * none failed). */
const char* rpca_last_error(const rpca_ctx* c);

/* Destroy a context (does not free the workspace or M). NULL is a no-op. */
void rpca_destroy(rpca_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* RPCA_H_ */
