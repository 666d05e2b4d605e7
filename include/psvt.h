/*
 * psvt -- singular value soft-thresholding through the polar decomposition,
 * on AMD Instinct MI355X (gfx950).
 *
 * Operation (section 2 of the paper, Eq. (1)): for A = U Sigma V^T,
 *     A_tau = U max(Sigma - tau I, 0) V^T.
 * Proposition 1 computes it without an SVD: with P = polar(A) and
 * S = polar(A^T A - tau^2 I),  A_tau = (A + A S)/2 - tau/2 (P + P S),
 * or, from the footnote, with S = polar(A A^T - tau^2 I),
 *     A_tau = (S A + A)/2 - tau/2 (S P + P).
 * (The proposition prints the shift as tau I; the proof requires
 * sign(sigma^2 - c) = sign(sigma - tau), i.e. c = tau^2, and the paper's code
 * listing shifts by tau**2.  This library shifts by tau^2.)
 * Both polar factors come from matmul-only odd-quintic iterations
 * (Newton-Schulz / Polar-Express type, sections 1 and 3).  The library
 * evaluates the proposition in the fused form A_tau = (A - tau P)(I + S)/2,
 * which is the same expression regrouped.
 *
 * Conventions for every entry point
 *   - Matrices are float32, row-major; ld* is the row stride in elements and
 *     must be >= the column count.  Matrix pointers are DEVICE pointers owned
 *     by the caller; inputs are read only, outputs are written only.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on `stream` and returns: no host synchronisation, no device
 *     allocation, no device-to-host read.  Results are ready when the stream
 *     reaches that point.  (psvt_svt with min(m, n) <= 2048 runs the polar
 *     iterations of P on a library-owned side stream of the calling thread,
 *     forked from `stream` and joined back into it by events before the
 *     final product.)
 *   - `ws` is caller-owned device scratch of at least psvt_workspace_bytes()
 *     bytes, 256-byte aligned; its contents need not be initialised and are
 *     garbage afterwards.  Calls that overlap in time must not share `ws`.
 *   - `cfg` may be NULL (all defaults).  A zero-initialised psvt_config means
 *     defaults too.
 *   - Return value: PSVT_OK or a negative PSVT_E* code; the argument checks
 *     run on the host before anything is enqueued, so on error nothing was
 *     launched.  psvt_last_error() gives a thread-local message.
 *   - m == 0 or n == 0 is a valid no-op.
 *   - Outputs must not overlap inputs or `ws` (PSVT_EINVAL when they do).
 */
#ifndef PSVT_H
#define PSVT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PSVT_OK = 0,
    PSVT_EINVAL = -1,       /* bad argument */
    PSVT_EWORKSPACE = -2,   /* ws NULL or smaller than psvt_workspace_bytes() */
    PSVT_EUNSUPPORTED = -3, /* current device is not gfx950 */
    PSVT_EHIP = -4          /* a HIP call or kernel launch failed */
};

/* operation ids for psvt_workspace_bytes */
enum { PSVT_OP_SVT = 0, PSVT_OP_POLAR = 1, PSVT_OP_POLAR_SYM = 2, PSVT_OP_RANK_R = 3 };

/* psvt_config.flags.
 *
 * Low-precision operands.  A BF16 iteration by default uses "split bf16"
 * operands (x = hi + lo, two bf16 planes, products hi.hi + hi.lo + lo.hi:
 * three bf16 MFMA passes, about 16 mantissa bits) for both polar factors:
 *   - S works on A^T A - tau^2 I, whose spectrum is the square of A's, so
 *     the eigenvalues that decide the sign sit far below bfloat16 resolution
 *     of the largest one;
 *   - the error of P enters A_tau multiplied by tau / (sigma - tau), which
 *     is up to 20 for singular values 5 % above tau.
 * With split operands the 18 BF16 + 2 FP32 schedule stays within 1e-2 of
 * the exact A_tau on inputs whose singular values keep a 5 % gap from tau.
 *   PSVT_FLAG_PLAIN_P  P's BF16 iterations use plain bf16 operands (one MFMA
 *                      pass).  Faster; the result then carries P's bf16
 *                      rounding times tau / (sigma - tau): measured up to
 *                      8e-2 for tau mid-spectrum with a 5 % gap, about 1e-3
 *                      for tau near the smallest singular values.
 *   PSVT_FLAG_PLAIN_S  S's BF16 iterations use plain bf16 operands (loses
 *                      the eigenvalues that decide the sign; not for
 *                      accuracy below 1e-1).
 *   PSVT_FLAG_SPLIT_P  accepted for compatibility: split P is the default.
 *   PSVT_FLAG_HFORM    (svt only) the H-form of the sign: with P = polar(A)
 *                      = U V^T, P^T A = V Sigma V^T, so (proof of
 *                      Proposition 1) S = sign(P^T A - tau I) = V1 V1^T -
 *                      V2 V2^T, the same S as sign(A^T A - tau^2 I) but on a
 *                      spectrum linear in sigma instead of squared.  The
 *                      iterations of S then run after P's (one more
 *                      product, P^T A); the shift tau is applied to the
 *                      diagonal in FP64.  Operand precision follows the
 *                      flags above; with PSVT_FLAG_PLAIN_S (plain bf16 S,
 *                      one MFMA pass instead of three) the H-form measures
 *                      0.9 - 1.5e-2 with 18 bf16 iterations, against 1.2e-1
 *                      for plain S on the squared spectrum.  S is built
 *                      from P, whose rotation error enters it multiplied by
 *                      sigma_max / (sigma - tau): the H-form takes no FP8
 *                      iterations (n_fp8 > 0 is PSVT_EINVAL).
 * FP8 iterations (n_fp8) use plain e4m3 operands in P and split bf16 in S.
 * K iterations with plain operands of unit roundoff u (2^-8 bf16, 2^-4
 * e4m3) leave polar() accurate to about u kappa sqrt(K) in the relative
 * Frobenius norm, kappa = sigma_max / sigma_min of the input: each such
 * iteration's rounding is amplified by sigma_max / sigma in the direction of
 * sigma, and the K contributions add up (measured: 18 plain bf16
 * iterations 2.0e-2 at kappa = 4; 6 e4m3 iterations 0.2 at kappa = 100).  In svt that error enters multiplied by
 * tau / (sigma - tau) on the retained directions, so the FP8 schedule suits
 * inputs whose retained singular values sit far above tau (low rank plus
 * noise), not tau inside a dense spectrum.
 *
 * Status word.  PSVT_FLAG_STATUS: the call also writes *psvt_config.status
 * (a caller-owned uint32_t in DEVICE memory, written on `stream` after the
 * output): a bit set of PSVT_STATUS_*.  It costs one norm pass over the
 * output and, for svt / rank_r / polar_sym, one symmetric s x s product
 * that measures the sign iteration's convergence:
 *   PSVT_STATUS_NONFINITE_INPUT   ||input||_F (FP64) is not finite;
 *   PSVT_STATUS_NONFINITE_OUTPUT  the output has a non-finite entry;
 *   PSVT_STATUS_NOT_CONVERGED     ||S^2 - I||_F / sqrt(s) > status_tol for
 *                                 the final sign iterate S (svt, rank_r,
 *                                 polar_sym; S^2 = I exactly when
 *                                 converged).  A singular shifted Gram
 *                                 (tau equal to a singular value, or
 *                                 tau = 0 with a rank-deficient input) also
 *                                 sets it. */
#define PSVT_FLAG_PLAIN_S 0x1u
#define PSVT_FLAG_SPLIT_P 0x2u
#define PSVT_FLAG_PLAIN_P 0x4u
#define PSVT_FLAG_STATUS 0x8u
#define PSVT_FLAG_HFORM 0x10u
/* psvt_svt_batched / psvt_rank_r_batched only: run the batch as ONE
 * persistent launch (below); PSVT_EINVAL elsewhere. */
#define PSVT_FLAG_PERSISTENT 0x20u
/* svt only: the polar factor in Gram form (for l >> s).  With T = X^T X,
 * every polar iterate is X N_k for a polynomial N_k in T, so the iteration
 * runs on s x s matrices only (Q = p(Y), N <- N Q, Y <- Y Q^2, on
 * Y0 = Pi T Pi / theta^2 + I - Pi with Pi = (I + S)/2 from the sign
 * iterations, which run first: the directions Pi removes are set to 1, so
 * N stays below sigma_max / tau; four s x s products per iteration, each
 * symmetrised, or 8 s^3 flops against 3 l s^2 + s^3 on the l x s iterate:
 * it pays for l >= 3 s), and A_tau = X (nu I - tau T^{-1/2}) (I + S)/2
 * takes one s x s and one l x s x s product (proof of Proposition 1:
 * A - tau P = A (I - tau (A^T A)^{-1/2})).  The P-side products are FP32
 * whatever the schedule (S follows it).  T squares the condition number of
 * the kept part: the error grows with sigma_max / tau (simulated in FP32:
 * about 3e-8 for low rank plus noise; 2e-6 to 1.3e-4 for log-spaced
 * spectra with sigma_max / tau from 3 to 4000).  Excludes PSVT_FLAG_HFORM. */
#define PSVT_FLAG_GRAM 0x40u

#define PSVT_STATUS_NONFINITE_INPUT 0x1u
#define PSVT_STATUS_NONFINITE_OUTPUT 0x2u
#define PSVT_STATUS_NOT_CONVERGED 0x4u
#define PSVT_STATUS_INVALID 0x8u /* batched: descriptor rejected on the device, matrix skipped */

/* side selection (Proposition 1 and its footnote) */
enum { PSVT_SIDE_AUTO = 0, PSVT_SIDE_RIGHT = 1, PSVT_SIDE_LEFT = 2 };

typedef struct psvt_config {
    /* Polar iterations per polar factor (the paper recommends 20, section 3;
     * its listing defaults to 11).  0 means 20.  Range 1..256. */
    int32_t iters;
    /* Precision schedule: the first n_fp8 iterations use FP8 (OCP e4m3)
     * operands, the next n_bf16 use BF16 operands, the rest FP32; all
     * accumulate in FP32 and keep an FP32 iterate.  n_fp8 + n_bf16 <= iters.
     * The Gram matrix and the final product are always FP32. */
    int32_t n_fp8;
    int32_t n_bf16;
    /* PSVT_SIDE_AUTO follows the paper's listing: right-sided (A^T A) when
     * n < m, else left-sided (A A^T). */
    int32_t side;
    /* Optional host array of iters x 3 quintic coefficients (a, b, c) that
     * replaces the built-in schedule (the paper's listing lets the caller
     * inject the polar algorithm).  Read during the call only. */
    const double *coeffs;
    /* PSVT_FLAG_* bits; 0 = defaults. */
    uint32_t flags;
    int32_t reserved0;
    /* Safety factor on the spectral bounds that scale each iterate into
     * the iteration's convergence region: the iterations start from
     * X / (norm_safety * theta), theta = sqrt(||X^T X||_F) >= sigma_max(X).
     * theta is already an upper bound (the built-in schedule tolerates 30 %
     * overshoot), so the default 1 suffices for it; a caller-supplied
     * schedule designed without margin may ask for more.  0 means 1;
     * otherwise in [1, 16]. */
    double norm_safety;
    /* PSVT_FLAG_STATUS: device pointer to the caller's status word. */
    uint32_t *status;
    /* Convergence threshold of PSVT_STATUS_NOT_CONVERGED on the RMS
     * deviation ||S^2 - I||_F / sqrt(s); 0 means 1e-3. */
    double status_tol;
    /* Warm start of the sign iteration (svt, rank_r), for a sequence of
     * thresholdings of slowly changing inputs such as the iterates of a
     * nuclear-norm proximal method (section 2).  pi_out (device, s x s,
     * row stride ld_pi; NULL = not written) receives this call's
     * Pi = (I + S)/2, s the side of the Gram matrix (n for right-sided
     * calls, m for left-sided ones).  warm_pi (device, s x s, ld_pi;
     * NULL = cold start) is a previous call's Pi for the same shape and
     * side: the sign iteration then starts from
     *     X0 = (H / theta + eps S_prev) / (1 + eps),  eps = 1e-3,
     * H the shifted Gram, theta its spectral bound, S_prev = 2 Pi - I, and
     * takes warm_iters (0 means 10) steps of the schedule instead of
     * `iters` (the last two in FP32, the others in split bf16 when the
     * schedule has low-precision iterations): every eigenvalue of X0 sits
     * at least about eps from 0, where the cold start has to amplify
     * eigenvalues down to |lambda| / theta.  H decides every direction with
     * |lambda| / theta >> eps, so an error carried by S_prev is damped by
     * about eps theta / |lambda| per call rather than accumulated; only a
     * direction with |lambda| / theta below about eps whose sign changed
     * since S_prev keeps the old sign, an error of at most |sigma - tau| in
     * that direction.  P's iterations are not warm started.  warm_pi and
     * pi_out may be the same buffer (read before written).  Not for
     * psvt_svt_batched. */
    const float *warm_pi;
    float *pi_out;
    int64_t ld_pi;
    int32_t warm_iters;
    int32_t reserved[3];
} psvt_config;

/* Workspace size for `op` on an m x n input (for PSVT_OP_POLAR_SYM, m = n). */
int psvt_workspace_bytes(int op, int64_t m, int64_t n, const psvt_config *cfg, size_t *bytes);

/* Y = A_tau (Eq. (1)) via Proposition 1.  A: m x n (lda), Y: m x n (ldy).
 * tau must be finite and >= 0.  tau = 0 gives A (up to the iterations'
 * accuracy); tau >= sigma_max gives 0. */
int psvt_svt(const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy, void *ws,
             size_t ws_bytes, const psvt_config *cfg, void *stream);

/* P = polar(A) = U V^T (section 2).  A: m x n (lda), P: m x n (ldp).  For a
 * rank-deficient A the iterations converge to the partial isometry over the
 * nonzero singular values. */
int psvt_polar(const float *A, int64_t m, int64_t n, int64_t lda, float *P, int64_t ldp, void *ws, size_t ws_bytes,
               const psvt_config *cfg, void *stream);

/* S = polar(G) for symmetric G, i.e. the matrix sign of its eigenvalues
 * (section 2).  G: n x n (ldg), symmetrised on load as (G + G^T)/2.
 * S: n x n (lds).  Zero eigenvalues map to 0. */
int psvt_polar_sym(const float *G, int64_t n, int64_t ldg, float *S, int64_t lds, void *ws, size_t ws_bytes,
                   const psvt_config *cfg, void *stream);

/* psvt_svt without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments as psvt_svt minus the workspace,
 * same kernels and results; the workspace is a static device array of
 * PSVT_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
 * on until the process ends (enough for every schedule up to 1024 x 1024;
 * larger problems return PSVT_EWORKSPACE).  Every launch goes to `stream`
 * (no side stream).  Calls that overlap in time on one device share the
 * array and race: serialise them (one stream, or events). */
#define PSVT_NOALLOC_SCRATCH_BYTES (96u << 20)
int psvt_svt_noalloc(const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy,
                     const psvt_config *cfg, void *stream);

/* Best rank-r approximation [A]_r (Corollary 1): with S = polar(A^T A -
 * tau^2 I), [A]_r = (A + A S)/2 = A (I + S)/2 (left-sided form for wide A).
 * tau must lie strictly between sigma_{r+1} and sigma_r (descending order). */
int psvt_rank_r(const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy, void *ws,
                size_t ws_bytes, const psvt_config *cfg, void *stream);

/* Batched form on a DEVICE array of descriptors: many svt (or rank_r)
 * problems of uneven shapes in one call that never reads the descriptors on
 * the host (the listing's batch note, section 4: leading batch dimensions;
 * here uneven shapes).  Nothing is allocated, nothing is synchronised and
 * nothing is read back: a setup kernel reads the descriptors, checks each
 * against the maximum shape, lays out its workspace inside `ws` and picks
 * its tile configurations with the library's cost model; then one launch
 * per stage of the method (products: one per tile configuration) processes
 * every matrix, each tile computed exactly as in a single call (results are
 * bitwise psvt_svt's / psvt_rank_r's).  The call may be captured into a HIP
 * graph and replayed; descriptors and inputs are read at run time, so their
 * contents may change between replays.
 *   d_descs  device array of `count` descriptors (0 <= count <= 2^20); each
 *            needs 1 <= m <= max_m, 1 <= n <= max_n, lda >= n, ldy >= n,
 *            non-NULL A and Y, tau finite and >= 0.  A descriptor that fails
 *            this is skipped (Y untouched); with PSVT_FLAG_STATUS its status
 *            word reads PSVT_STATUS_INVALID.
 *   status   per descriptor (device pointer or NULL): with PSVT_FLAG_STATUS
 *            in cfg the matrix's status word (psvt_config.status is not
 *            used); ignored otherwise.
 *   ws       device memory of psvt_batched_workspace_bytes(op, count,
 *            max_m, max_n, cfg) bytes (a bound over every shape within the
 *            maxima), 256-byte aligned, owned by the caller; calls that
 *            overlap in time must not share it.
 *   Errors are host-side checks of count, maxima, workspace and cfg (nothing
 *   is launched then).  Outputs must not overlap inputs, other outputs or
 *   ws (not checked: the shapes are on the device).
 *
 * PSVT_FLAG_PERSISTENT: after the setup kernels (the descriptor pass, a few
 * small kernels that copy the stage templates into ws, and one that lays out
 * the dependency counts), ONE launch of two blocks per CU runs every stage of
 * every matrix.  Blocks take tickets in the order of the per-stage launches
 * (stage by stage, matrices in order, tiles in order); an item of matrix i
 * waits until matrix i has completed all its items of earlier stages, so
 * small matrices run ahead of large ones and no stage drains the device.
 * Every wait is on an item with a lower ticket, held by a running block, so
 * the launch always drains; a wait is also bounded (about seconds,
 * psvt_tune_spin_limit): past the bound the block raises the abort flag,
 * every later item is skipped, the launch ends, the 32-bit word at byte 4
 * of ws reads nonzero and, with PSVT_FLAG_STATUS, status words read
 * PSVT_STATUS_INVALID for the matrices that did not finish.  The executor
 * holds tiles up to 128 x 128 (f32, bf16) and 64 x 64 (split bf16, fp8):
 * results are bitwise those of single calls made with
 * psvt_tune_persistent_tiles(1) on the calling thread.  The workspace is
 * larger (psvt_batched_workspace_bytes with the flag set). */
typedef struct psvt_desc {
    const float *A; /* m x n input, row-major, device */
    float *Y;       /* m x n output, row-major, device */
    int64_t m, n, lda, ldy;
    double tau;
    uint32_t *status;
} psvt_desc;
int psvt_batched_workspace_bytes(int op, int32_t count, int64_t max_m, int64_t max_n, const psvt_config *cfg,
                                 size_t *bytes);
int psvt_svt_batched(const psvt_desc *d_descs, int32_t count, int64_t max_m, int64_t max_n, void *ws,
                     size_t ws_bytes, const psvt_config *cfg, void *stream);
int psvt_rank_r_batched(const psvt_desc *d_descs, int32_t count, int64_t max_m, int64_t max_n, void *ws,
                        size_t ws_bytes, const psvt_config *cfg, void *stream);

/* Host-only replay of the persistent executor's schedule (for tests; no
 * device is touched): for `count` shapes ms[i] x ns[i] (host arrays) it
 * builds the tables the setup kernels would, checks that tickets map one to
 * one onto items, that each item's dependency count is its matrix's items of
 * earlier launches, and that `blocks` simulated blocks with random item
 * durations (xorshift from `seed`) drain every ticket without deadlock, no
 * item starting before its matrix's earlier launches completed.  *tickets =
 * the launch's ticket count.  PSVT_EINVAL with psvt_last_error() naming the
 * first violated check. */
int psvt_batched_check_schedule(int op, const int64_t *ms, const int64_t *ns, int32_t count, int64_t max_m,
                                int64_t max_n, const psvt_config *cfg, int32_t blocks, uint64_t seed,
                                int64_t *tickets);

/* Batched form from a HOST item array: many svt (or rank_r) problems of
 * uneven shapes, planned once on the host.
 *
 * psvt_batch_create plans the batch on the host: every item runs the same
 * stage list, and stage k of all items becomes grouped launches (products
 * grouped by the tile configuration the autotuned cost model picks for each
 * item's size, largest first, blocks mapped to (item, tile) through a prefix
 * sum).  It copies the descriptor tables to a device buffer it allocates, and
 * captures one run into a HIP graph; it synchronises and allocates, so call
 * it outside graph capture.  Items are read through their pointers at run
 * time, so their contents may change between runs.
 * psvt_batch_run enqueues the grouped launches on `stream`;
 * psvt_batch_run_graph replays the captured graph on `stream` (one graph
 * launch).  Neither allocates or synchronises.  Runs of one batch must not
 * overlap (they share `ws`).
 * `ws`: caller-owned device memory of psvt_batch_workspace_bytes(), 256-byte
 * aligned, that must outlive the batch.  op: PSVT_OP_SVT or PSVT_OP_RANK_R. */
typedef struct psvt_batch_item {
    const float *A; /* m x n input, row-major, device */
    float *Y;       /* m x n output, row-major, device */
    int64_t m, n, lda, ldy;
    double tau;
    /* per-item warm start (psvt_config.warm_pi / pi_out / ld_pi; NULL =
     * cold / not written); the configuration's own fields are not used */
    const float *warm_pi;
    float *pi_out;
    int64_t ld_pi;
} psvt_batch_item;
typedef struct psvt_batch psvt_batch;
int psvt_batch_workspace_bytes(int op, const psvt_batch_item *items, int32_t count, const psvt_config *cfg,
                               size_t *bytes);
int psvt_batch_create(int op, const psvt_batch_item *items, int32_t count, void *ws, size_t ws_bytes,
                      const psvt_config *cfg, psvt_batch **out);
int psvt_batch_run(psvt_batch *batch, void *stream);
int psvt_batch_run_graph(psvt_batch *batch, void *stream);
/* number of grouped launches per run and useful flops per run */
int psvt_batch_stats(const psvt_batch *batch, int32_t *launches, double *flops);
int psvt_batch_destroy(psvt_batch *batch);

/* Serving: a request loop for svt / rank_r calls of mixed sizes.
 *
 * A server owns a device memory pool of `budget_bytes` (the HBM budget) and
 * a worker thread.  Requests are admitted in arrival order while fewer than
 * `max_slots` are active and the pool has room for the request's workspace
 * (a request never overtakes an earlier one).  An admitted request's
 * iterates stay in its workspace on the device until it completes.
 * Admitted requests are split by size (s^2 l, s and l the short and long
 * side) into four lanes.  The worker runs ticks per lane: every active
 * request of the lane advances by up to 3 stages of its stage list (for a
 * short side <= 2048 by up to 3 stages of each of its P and S iteration
 * chains, which then have separate buffers, as in psvt_svt); a round's
 * stages are grouped by kind (products also by operand type and tile
 * configuration) into grouped launches, so requests at the same stage share
 * launches.  Newcomers start with the lane's next cohort (below), or at the
 * next tick with PSVT_SERVER_EAGER; either way requests enter and leave a
 * running lane without draining the server (continuous batching).  Each
 * lane has its own stream, so
 * lanes overlap on the device.  Tiles are computed exactly as in single
 * calls, so a result is the same alone and in the mix.  All requests use the
 * server's psvt_config (its coeffs are copied).
 *   create:  allocates the pool, the lanes' streams and descriptor rings;
 *            PSVT_SERVER_FAKE runs the scheduler without a device (stages
 *            complete at once; for tests).  Cohort admission (the default;
 *            PSVT_SERVER_COHORT asks for it explicitly): a request admitted
 *            while its lane runs requests that have started waits until they
 *            have launched their last stage, then starts with the other
 *            waiting ones, so a cohort's requests sit at the same stage and
 *            share launches.  PSVT_SERVER_EAGER: a request joins its lane's
 *            running requests at once instead (they then rarely share a
 *            stage).  Setting both is PSVT_EINVAL.
 *   submit:  non-blocking; A is read and Y written by the device at some
 *            later time, so both must stay valid until the request is done.
 *            `stream` is the caller's stream (hipStream_t, NULL = default)
 *            that produced A and last used Y: an event recorded on it at
 *            submit orders the request's first stage after that work (the
 *            request itself runs on the server's streams).  Results are
 *            ready once poll / wait report state 2 (done).
 *            PSVT_EWORKSPACE if the request could never fit the budget.
 *   poll / wait:  state 0 queued, 1 running, 2 done, -1 failed.
 *   drain:   waits until nothing is queued or active; returns the first
 *            launch error the server met, if any (requests of other ticks
 *            and lanes are not affected by it).
 *   stats:   latency = completion observed by the worker - submit time.
 * Failures stay with their requests: a request whose plan fails, whose
 * submitter event cannot be waited for, or that passes its deadline fails
 * alone; a launch error fails the requests of that tick (they share its
 * launches), and the lane goes on with its other requests.  The workspace
 * of a request failed while its stages may be in flight returns to the pool
 * once its lane's last tick has passed on the device.
 *   set_timeout:  a request not done `seconds` after its submit fails
 *            (state -1, counted in timed_out); 0 (the default) = none.
 *   inject_fault: PSVT_SERVER_FAKE servers only (tests of the failure
 *            paths): PSVT_FAULT_TICK fails the n-th tick (counted over all
 *            lanes from 0) as a launch error would; PSVT_FAULT_PLAN fails
 *            the n-th admission's plan; PSVT_FAULT_STALL with n != 0 stops
 *            fake ticks from completing, n = 0 lets them complete again. */
#define PSVT_SERVER_FAKE 0x1u
#define PSVT_SERVER_COHORT 0x2u
#define PSVT_SERVER_EAGER 0x4u
typedef struct psvt_server psvt_server;
enum { PSVT_FAULT_TICK = 1, PSVT_FAULT_PLAN = 2, PSVT_FAULT_STALL = 3 };
typedef struct psvt_server_counters {
    int64_t submitted, completed, failed, queued, active, ticks, launches;
    double p50_ms, p99_ms, max_ms, queue_p99_ms, matrices_per_s;
    size_t budget_bytes, peak_bytes;
    int64_t timed_out; /* failed requests that passed their deadline */
} psvt_server_counters;
int psvt_server_create(size_t budget_bytes, int32_t max_slots, const psvt_config *cfg, uint32_t flags,
                       psvt_server **out);
int psvt_server_submit(psvt_server *server, int op, const psvt_batch_item *item, void *stream, uint64_t *ticket);
int psvt_server_poll(psvt_server *server, uint64_t ticket, int32_t *state);
int psvt_server_wait(psvt_server *server, uint64_t ticket, double timeout_s, int32_t *state);
int psvt_server_drain(psvt_server *server, double timeout_s);
int psvt_server_stats(psvt_server *server, psvt_server_counters *stats);
int psvt_server_set_timeout(psvt_server *server, double seconds);
int psvt_server_inject_fault(psvt_server *server, int kind, int64_t n);
int psvt_server_destroy(psvt_server *server);

/* Building blocks exposed for kernel-level tests and tuning.
 *
 * psvt_gemm_nt: the MFMA product used by every step of the method,
 *     C[i][j] = alpha * sum_k A[i][k] B[j][k] + beta * D[i][j]
 * with A (M x K) and B (N x K) stored in `dtype` (PSVT_DTYPE_F32: float,
 * PSVT_DTYPE_BF16: bfloat16 bits, PSVT_DTYPE_FP8: OCP e4m3 bytes,
 * PSVT_DTYPE_BF16X3: split bfloat16, the hi plane followed by the lo plane,
 * each rows x ld, product hi.hi + hi.lo + lo.hi) and C, D
 * (M x N) float32; all row-major device buffers, 16-byte aligned, with every
 * row stride a multiple of 16 bytes.  Products accumulate in FP32.  D may be
 * NULL.  sym != 0 requires M == N and computes only the lower block
 * triangle, mirroring it into the upper one (valid when the product is
 * symmetric, e.g. A = B).
 *
 * psvt_convert: Y = round(scale * X) into `dtype` (bfloat16: round to
 * nearest even; FP8 e4m3: round to nearest even, saturated to +-448; split
 * bfloat16: hi = bf16(x) then lo = bf16(x - hi) in a second plane), or
 * into float32 when dtype is PSVT_DTYPE_F32; transpose != 0 writes
 * Y[j][i] instead of Y[i][j].  X: rows x cols float32 (ldx), Y: ldy in
 * elements of `dtype`. */
int psvt_gemm_nt(int dtype, const void *A, int64_t lda, const void *B, int64_t ldb, const float *D, int64_t ldd,
                 float *C, int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta, int sym,
                 void *stream);
int psvt_convert(int dtype, const float *X, int64_t rows, int64_t cols, int64_t ldx, void *Y, int64_t ldy,
                 float scale, int transpose, void *stream);

/* Launch tracing.  psvt_trace_begin() starts recording every kernel launch
 * that the library makes from the calling thread: each is bracketed by two
 * HIP events recorded on the launch's stream (so the elapsed time is device
 * time of that launch alone).  psvt_trace_end() waits for the recorded
 * events (a host synchronisation), aggregates them per kernel name, most
 * time first, writes up to max_entries rows to `out` and stops recording.
 * `flops` are useful flops (a symmetric product counts half), `bytes` the
 * algorithmic HBM bytes of memory-bound kernels (0 for products).  Names are
 * static strings.  Meant for profiling: the events add a few microseconds
 * per launch. */
typedef struct psvt_trace_stat {
    const char *name;
    int64_t launches;
    double total_ms;
    double flops;
    double bytes;
} psvt_trace_stat;
int psvt_trace_begin(void);
int psvt_trace_end(psvt_trace_stat *out, int max_entries, int *n_entries);

/* Tile configurations of the MFMA kernels.  Ids: 1 = 64x64 tiles (4 blocks
 * per CU; 2 for split bf16), 2 = 128x128 (2 per CU; 1 for split bf16),
 * 3 = 192x192 (1 per CU), 4 = 256x256 (1 per CU).  Each product picks the configuration with the smallest
 * modelled time
 *     (most tiles on one CU) x (overhead + tile flops / (eff x CU rate)),
 * with (eff, overhead) per operand dtype (PSVT_DTYPE_*; for split bf16 the
 * CU rate is a third of bf16's, so eff is per useful flop), kind (sym = 1 for
 * the lower-triangle products, 0 for full ones) and configuration, measured
 * by the autotuner.
 *   psvt_tune_force_tile(id)   force a configuration on the calling thread
 *                              (0 = automatic).
 *   psvt_tune_set(dtype, id, sym, eff, overhead_us)  eff in (0, 1],
 *                              overhead >= 0 microseconds.
 *   psvt_tune_load(path)       read "dtype id sym eff overhead_us" lines ('#'
 *                              starts a comment); PSVT_EINVAL on a malformed
 *                              line, and then nothing is applied.
 *   psvt_tune_pick             the id the model picks for an M x N x K
 *                              product (>= 1), or a negative error code.
 *   psvt_tune_persistent_tiles(on)  single calls on the calling thread pick
 *                              from the persistent executor's tile set
 *                              (PSVT_FLAG_PERSISTENT), so that they compute
 *                              every tile as it does (1 = on, 0 = off).
 *   psvt_tune_spin_limit(n)    the calling thread's bound on one dependency
 *                              wait of the persistent executor, in polls
 *                              (about a microsecond each; default 2^22,
 *                              0 = abort on any wait that is not already
 *                              satisfied: a test of the abort path).
 * The model is process-wide; change it before concurrent calls. */
enum { PSVT_DTYPE_F32 = 0, PSVT_DTYPE_BF16 = 1, PSVT_DTYPE_FP8 = 2, PSVT_DTYPE_BF16X3 = 3 };
int psvt_tune_force_tile(int tile);
int psvt_tune_set(int dtype, int tile, int sym, double efficiency, double overhead_us);
int psvt_tune_load(const char *path);
int psvt_tune_pick(int dtype, int64_t M, int64_t N, int64_t K, int sym);
int psvt_tune_persistent_tiles(int on);
int psvt_tune_spin_limit(int64_t polls);

/* Static description of a return code. */
const char *psvt_strerror(int code);

/* Thread-local detail of the last failing call on this thread ("" if none). */
const char *psvt_last_error(void);

/* Library version string. */
const char *psvt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PSVT_H */
