/*
 * ciq.h -- C ABI of libciq: msMINRES-CIQ matrix square roots on MI355X (gfx950).
 *
 * Method: Pleiss, Jankowiak, Eriksson, Damle, Gardner, "Fast Matrix Square
 * Roots with Applications to Gaussian Processes and Bayesian Optimization"
 * (NeurIPS 2020). For a kernel matrix
 *
 *     K = o^2 k(X, X) + sigma^2 I,      k = RBF or Matern-5/2 (isotropic or ARD)
 *
 * the library computes K^{-1/2} B and K^{1/2} B through the rational
 * approximation of Sec. 3 (K^{-1/2} ~= sum_q w_q (t_q I + K)^{-1}), the
 * Hale-Higham-Trefethen shifts/weights of Appendix B (Alg. S2) and one
 * multi-shift MINRES run (Appendix C, Alg. S4) whose Lanczos recurrence shares
 * a single kernel product K V per iteration across all Q shifts. Products
 * regenerate K's entries from X, or stream a copy of K that the call writes
 * once and frees (ciq_opts.kernel_cache). An optional pivoted-Cholesky
 * preconditioner (Sec. 3.4, Appendix D; ciq_opts.precond_rank) gives results
 * equal to K^{+-1/2} B up to an orthogonal rotation in fewer iterations. The
 * same engine serves the paper's applications: posterior covariance roots
 * for Thompson sampling (ciq_posterior_mvm, Sec. 5.2), sparse operators such
 * as a Gibbs sampler's precision (ciq_csr_mvm, Sec. 5.3) and the whitened
 * SVGP predictive pass (ciq_svgp_predict, Sec. 5.1, App. E).
 *
 * Conventions shared by every entry point:
 *  - Status: every call returns CIQ_OK (0) or one of the CIQ_E* codes below;
 *    ciq_strerror() names it. Arguments are validated before any device work:
 *    on CIQ_EINVAL nothing has been launched and no output was written.
 *  - Memory: X, B, V, Y, out, solves, G, dB are caller-owned DEVICE buffers,
 *    row-major with the stated leading dimension (in elements). Inputs are not
 *    modified. Lengthscales, t/w tables, info and gradient scalars are HOST
 *    memory. The library keeps a grow-only scratch area per device (freed at
 *    process exit); calls on one device are serialised by an internal lock.
 *  - Streams: work is queued on `stream` (0 = the null stream). Solver calls
 *    (eig_bounds, sqrt/invsqrt, backward, batched) poll convergence and return
 *    only after their work on `stream` has completed; ciq_kernel_mvm returns
 *    immediately (asynchronous on `stream`).
 *  - Element types: dtype CIQ_F64 uses double for X, B, V, Y, out, solves, G
 *    and dB; every other dtype uses float for them. Lanczos/Givens scalars,
 *    reductions, shifts, weights and eigenvalue bounds are always double.
 *  - Non-convergence is not an error: see ciq_info.converged.
 */
#ifndef CIQ_H
#define CIQ_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CIQ_OK        0
#define CIQ_EINVAL    1   /* bad argument (null pointer, size <= 0, bad enum, ...) */
#define CIQ_ENOMEM    2   /* device scratch allocation failed                        */
#define CIQ_EHIP      3   /* a HIP runtime call failed                               */
#define CIQ_ENOTSUP   4   /* valid request this build does not implement             */
#define CIQ_ENUMERIC  5   /* NaN/Inf met in the Lanczos scalars                      */

/* ---- enums --------------------------------------------------------------- */
#define CIQ_KERNEL_RBF       0   /* k = exp(-r^2/2)                                  */
#define CIQ_KERNEL_MATERN52  1   /* k = (1 + sqrt5 r + 5 r^2/3) exp(-sqrt5 r)        */
/* r^2 = sum_d (x_d - x'_d)^2 / l_d^2; l isotropic (1 value) or ARD (d values)      */

#define CIQ_F64     0   /* double everywhere; FP64 entries, FP64 MFMA contraction    */
#define CIQ_F32     1   /* float inputs/outputs; FP32 entries, FP32 MFMA contraction
                           (FP64 running sums); FP64 Krylov vectors and scalars.
                           With a resident K, K^{-1/2}B solves of at most 32
                           columns contract the FP32 entries on the FP64 MFMA
                           (no FP32 sums: the result is the rounded matrix's),
                           wider ones keep FP32 sums of 16 columns; K^{1/2}B
                           solves keep FP32 sums of 16 (<= 32 columns) or 64
                           columns, which its final product with K damps      */
#define CIQ_BF16X3  2   /* as CIQ_F32, but the entries and V are split into BF16
                           hi + scaled lo parts: K V ~ Kh Vh + 2^-8 (Kh Vl + Kl Vh)
                           on bf16 MFMA, FP32 accumulation (~1e-5 per product)   */
#define CIQ_F16X3   3   /* the same split in FP16 (lo parts scaled by 2^11),
                           ~1e-6 per product on the fly; with a resident K
                           (ciq_opts.kernel_cache) the FP64 entries are stored
                           split once, hi + 2^-11 lo (4 bytes per entry), and
                           three part products run on FP16 MFMA (~1e-7 per
                           product, FP32-class); ciq_backward and the batched
                           call return CIQ_ENOTSUP for both split forms        */

#define CIQ_INVSQRT 0
#define CIQ_SQRT    1

#define CIQ_BASIS_AUTO 0
#define CIQ_BASIS_OFF  1

#define CIQ_CACHE_AUTO 0   /* keep K resident when it fits (see ciq_opts.kernel_cache) */
#define CIQ_CACHE_OFF  1   /* evaluate kernel entries in every product                */
#define CIQ_CACHE_ON   2   /* always keep K resident (CIQ_ENOMEM if it does not fit)  */

#define CIQ_MAX_Q   64   /* quadrature points                                       */
#define CIQ_MAX_D   16   /* input dimensions                                        */
#define CIQ_MAX_RANK 1024 /* preconditioner rank                                    */
#define CIQ_MAX_OBS  4096 /* observations of ciq_posterior_mvm                       */
#define CIQ_NOALLOC_SCRATCH_BYTES (64u << 20) /* static scratch of ciq_kernel_mvm_noalloc */

/* One kernel matrix K = outputscale * k(X, X) + noise * I. */
typedef struct ciq_problem {
    int32_t n;                 /* points (rows of X), >= 1                         */
    int32_t d;                 /* input dimensions, 1..CIQ_MAX_D                   */
    const void* x;             /* device, n x d row-major (ld = d), see dtype       */
    int32_t kernel;            /* CIQ_KERNEL_*                                      */
    int32_t n_lengthscale;     /* 1 (isotropic) or d (ARD)                          */
    const double* lengthscale; /* host, n_lengthscale values > 0                    */
    double outputscale;        /* o^2 > 0                                           */
    double noise;              /* sigma^2 >= 0 (diagonal only)                      */
} ciq_problem;

/* A sparse symmetric matrix in CSR form (device arrays, FP64 values). */
typedef struct ciq_csr {
    int32_t n;                 /* rows = columns, >= 1                              */
    int32_t nnz;               /* stored entries                                    */
    const int32_t* row_ptr;    /* device, n + 1 offsets into col_idx / val          */
    const int32_t* col_idx;    /* device, nnz column indices (0-based)              */
    const double* val;         /* device, nnz values                                */
} ciq_csr;

/* Solver options. Zero-initialise and set what you need. */
typedef struct ciq_opts {
    int32_t dtype;             /* CIQ_F64 / CIQ_F32 / CIQ_BF16X3 / CIQ_F16X3        */
    int32_t q;                 /* quadrature points Q, 1..CIQ_MAX_Q                 */
    int32_t max_iter;          /* msMINRES iteration cap J (= products with K)      */
    double tol;                /* stop shift q of column s when
                                  |phibar|/||b_s|| <= tol (tol >= 0)                */
    int32_t lanczos_steps;     /* Lanczos steps for the eigenvalue bounds (0 -> 20) */
    uint64_t seed;             /* seed of the bounds' start vector (SplitMix64)     */
    double lambda_min;         /* if lambda_min > 0 and lambda_max >= lambda_min:  */
    double lambda_max;         /*   use these bounds, skip the Lanczos estimate     */
    int32_t check_every;       /* iterations between host convergence polls (0: auto) */
    int32_t profile;           /* 1: time every kernel-product launch of the msMINRES
                                  loop with HIP events on `stream` (ciq_info.mvm_ms) */
    int32_t kernel_cache;      /* CIQ_CACHE_*. Single-problem CIQ_F64 / CIQ_F32 /
                                  CIQ_F16X3 solves (and ciq_backward) may write the
                                  unit-scale entries k(x_i, x_j) once per call into a
                                  device buffer of ceil(n/128)*128 x ceil(n/64)*64
                                  doubles (CIQ_F64, 20 GB at n = 50,000), floats
                                  (CIQ_F32, entries evaluated in FP64 and rounded
                                  once) or FP16 hi/lo pairs (CIQ_F16X3, 4 bytes per
                                  entry) and stream them in every product instead of
                                  re-evaluating them; the buffer is allocated and
                                  freed inside the call. The batched call (FP32)
                                  keeps one such FP32 matrix per problem (their
                                  total must fit the same way). CIQ_BF16X3
                                  ignores this field.                            */
    int32_t cache_budget_mib;  /* CIQ_CACHE_AUTO: largest matrix kept, in MiB
                                  (0: half of the free device memory at the call) */
    int32_t graph;             /* 1: capture two msMINRES iterations (all their
                                  kernels) once in a HIP graph and replay it, one
                                  launch per two iterations (small problems are
                                  launch-bound); ignored with profile = 1. The
                                  arithmetic is the same as without it.         */
    int32_t precond_rank;      /* R > 0: pivoted-Cholesky preconditioned msMINRES-CIQ
                                  (Sec. 3.4, Appendix D), single-problem calls only,
                                  needs noise > 0, R <= CIQ_MAX_RANK (clamped to n).
                                  P = Lbar Lbar^T + sigma^2 I with Lbar the rank-R
                                  factor of ciq_pivoted_cholesky; the solves run on
                                  P^{-1/2} K P^{-1/2} (P^{-1} by the inversion lemma,
                                  P^{1/2} B in closed form from the eigenvalues of
                                  Lbar^T Lbar), and the outputs are
                                    invsqrt: R' B = P^{-1/2} (P^{-1/2} K P^{-1/2})^{-1/2} B
                                    sqrt:    R B = K R' B
                                  with R' R'^T = K^{-1} and R R^T = K: K^{-1/2} B and
                                  K^{1/2} B up to an orthogonal rotation (the same
                                  rotation for every column), not those matrices
                                  themselves. The eigenvalue bounds, tol and
                                  max_rel_residual refer to the preconditioned
                                  system. 0: plain CIQ. ciq_backward and the batched
                                  call return CIQ_ENOTSUP for R > 0.             */
    int32_t krylov_basis;      /* CIQ_BASIS_AUTO: when the run has neither a
                                  preconditioner nor kept per-shift solves and
                                  (max_iter + 1) Lanczos vectors fit in device
                                  memory, keep the vectors the run reaches
                                  resident and form the solution once after the
                                  run from the logged direction coefficients,
                                  instead of moving Q direction vectors every
                                  iteration (the same result up to rounding).
                                  The vectors live in 2 GiB chunks
                                  ($CIQ_BASIS_CHUNK_MIB sets another size) that
                                  stay allocated on the device after the call
                                  for the next one (ciq_release_workspace
                                  returns them); a chunk the device cannot
                                  supply in the middle of a run ends it with
                                  CIQ_ENOMEM.
                                  CIQ_BASIS_OFF: the direction recurrence.       */
    int32_t reserved;
} ciq_opts;

/* Per-call report (host). Valid when the call returned CIQ_OK. */
typedef struct ciq_info {
    int32_t iters;             /* products with K in the msMINRES run               */
    int32_t converged;         /* 1 if every (shift, column) met tol               */
    int32_t q;                 /* quadrature points used                           */
    int32_t mvm_count;         /* all products with K in the call (bounds included) */
    double max_rel_residual;   /* max over (q, s) of |phibar|/||b_s||              */
    double lambda_min;         /* bounds the quadrature was built on               */
    double lambda_max;
    double t[CIQ_MAX_Q];       /* shifts t_q (ascending)                           */
    double w[CIQ_MAX_Q];       /* weights w_q                                      */
    double mvm_ms;             /* opts.profile: summed device time of the timed
                                  kernel-product launches (ms), else 0             */
    int32_t mvm_timed;         /* number of launches in mvm_ms                     */
    int32_t kernel_cached;     /* 1 if the products streamed a resident K           */
    int32_t precond_rank;      /* pivots the preconditioner's factor took (<= R), 0
                                  without preconditioning                           */
    double precond_trace;      /* trace of o^2 k(X, X) - Lbar Lbar^T (0 without)    */
    double setup_ms;           /* host wall time (ms) of the preconditioner's or the
                                  posterior's factors, built before the Krylov runs
                                  (0 when the call has neither)                     */
    int32_t krylov_basis;      /* 1 if the run kept its Lanczos basis resident       */
} ciq_info;

/* Library version (major*10000 + minor*100 + patch). */
int ciq_version(void);

/* Name of a status code (static string, never NULL). */
const char* ciq_strerror(int status);

/*
 * Frees the device memory the library keeps on `device` between calls: the
 * chunks of the resident Krylov basis and their coefficient logs
 * (ciq_opts.krylov_basis), and the grow-only iteration scratch. Later calls
 * allocate again what they need. The library also returns the basis chunks by
 * itself when a later allocation would not fit beside them. Waits for a call
 * running on that device in another thread to end, then for the device to
 * drain. Leaves the current device unchanged.
 * Errors: CIQ_EINVAL for a device index out of range; CIQ_EHIP if the runtime
 * fails.
 */
int ciq_release_workspace(int device);

/*
 * Hale-Higham-Trefethen quadrature for K^{-1/2} on [lambda_min, lambda_max]
 * (Appendix B, nodes/weights formula with t_q = -sigma_q^2, w_q = -w~_q; Alg. S2
 * with k'^2 = 1 - k^2). Host-only FP64; Jacobi sn/cn/dn by the AGM / descending
 * Landen method and K' = pi / (2 AGM(1, k)) (Abramowitz & Stegun 16.4, 17.6),
 * so 1 - k^2 is never formed.
 *   t_out, w_out: caller-owned host arrays of length q; t ascending, all > 0; w > 0.
 * Errors: CIQ_EINVAL unless 0 < lambda_min <= lambda_max < inf, 1 <= q <= CIQ_MAX_Q
 * and both outputs are non-NULL.
 */
int ciq_setup(double lambda_min, double lambda_max, int q, double* t_out, double* w_out);

/*
 * Y = K V for the s columns of V (the on-the-fly kernel product of Sec. 3.2 and
 * Property 1; K is generated tile by tile and never stored).
 *   v: device, n x s, leading dimension ldv >= s; y: device, n x s, ldy >= s.
 *   dtype selects the element type and the contraction (see CIQ_F64..CIQ_F16X3).
 * Asynchronous on `stream`. Errors: CIQ_EINVAL on bad sizes/pointers/enums.
 */
int ciq_kernel_mvm(const ciq_problem* p, int dtype, const void* v, int s, int ldv,
                   void* y, int ldy, hipStream_t stream);

/*
 * ciq_kernel_mvm without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and launch configuration, with the
 * scaled points and the FP64 split partials in a static device array of
 * CIQ_NOALLOC_SCRATCH_BYTES per GPU (reserved when the library is loaded,
 * held until the process ends) instead of stream-ordered allocations.
 * Results equal ciq_kernel_mvm's. Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (different streams or host threads
 * without ordering) race and give wrong results; calls on one stream are
 * ordered. The caller still supplies v and y.
 * Asynchronous on `stream`. Errors: as for ciq_kernel_mvm, and CIQ_EINVAL when
 * n * d_pad * 8 (rounded up to 256) + nsplit * n * s * 8 bytes exceed
 * CIQ_NOALLOC_SCRATCH_BYTES (d_pad: d padded to 4/6/8/10/12/16; nsplit <= 8,
 * the split of the column range the kernel uses; CIQ_F64 with one split and
 * s <= 64 needs no partials); CIQ_EHIP if the array's address cannot be taken.
 */
int ciq_kernel_mvm_noalloc(const ciq_problem* p, int dtype, const void* v, int s, int ldv,
                           void* y, int ldy, hipStream_t stream);

/*
 * Y = K V by the resident-matrix product the solvers use when
 * ciq_opts.kernel_cache keeps K in device memory (Sec. 3.2): the unit-scale
 * entries are written once into a buffer allocated for this call, then the
 * product kernel runs once with the launch configuration a solve of this n
 * and s uses, and the buffer is freed. dtype: CIQ_F64 (FP64 entries, FP64
 * MFMA), CIQ_F32 (FP64 entries rounded once to FP32, FP32 MFMA, FP32 sums
 * of 16 or 64 columns as a K^{1/2}B solve runs them, FP64 beyond), CIQ_F16X3
 * (FP64 entries split into FP16
 * hi + 2^-11 lo, V split likewise after a per-column power-of-two scale,
 * three part products on FP16 MFMA); CIQ_BF16X3 is CIQ_ENOTSUP.
 *   v, s, ldv, y, ldy: as for ciq_kernel_mvm.
 * Synchronous. Errors: as for ciq_kernel_mvm; CIQ_ENOMEM if the matrix does not
 * fit; CIQ_ENOTSUP for CIQ_BF16X3.
 */
int ciq_kernel_mvm_resident(const ciq_problem* p, int dtype, const void* v, int s, int ldv,
                            void* y, int ldy, hipStream_t stream);

/*
 * Extreme-eigenvalue estimate of K (Appendix B.2; Alg. S2 first step): `steps`
 * Lanczos steps (0 -> 20) from v0 (device, n values; NULL -> a SplitMix64 draw
 * from `seed`), eigenvalues of T by cyclic Jacobi on the host, widened as
 *   lambda_max = theta_max + beta_{J+1} |y_J(theta_max)|   (Ritz residual),
 *   lambda_min = min(theta_min, sigma^2) if sigma^2 > 0, else theta_min / 2.
 * Outputs are host doubles. Synchronous.
 */
int ciq_eig_bounds(const ciq_problem* p, int dtype, int steps, const void* v0,
                   uint64_t seed, double* lambda_min, double* lambda_max,
                   hipStream_t stream);

/*
 * out = K^{-1/2} B (ciq_invsqrt_mvm) or K^{1/2} B (ciq_sqrt_mvm) by msMINRES-CIQ
 * (Alg. S1; the square root multiplies the weighted solve sum by K once more,
 * Sec. 3 rational approximation).
 *   b: device n x s (ldb >= s); out: device n x s (ldo >= s).
 *   solves: NULL, or device [n][q][s] (contiguous) receiving the per-shift
 *     solutions x^{(q)} ~= (t_q I + K)^{-1} b, as needed by ciq_backward.
 *   info: host, required.
 * Stopping: per (shift, column) at |phibar|/||b_s|| <= tol, frozen thereafter;
 * all at max_iter. A zero column of B gives a zero output column.
 * Synchronous. Errors: CIQ_EINVAL (n, s, q, max_iter, tol, pointers, ldb/ldo,
 * dtype/kernel/d out of range), CIQ_ENOMEM, CIQ_EHIP, CIQ_ENUMERIC.
 */
int ciq_invsqrt_mvm(const ciq_problem* p, const ciq_opts* o, const void* b, int s, int ldb,
                    void* out, int ldo, void* solves, ciq_info* info, hipStream_t stream);
int ciq_sqrt_mvm(const ciq_problem* p, const ciq_opts* o, const void* b, int s, int ldb,
                 void* out, int ldo, void* solves, ciq_info* info, hipStream_t stream);

/*
 * Vector-Jacobian product of a forward call made with the same p, shifts t/w
 * (from its ciq_info) and its saved `solves` (Sec. 3.3):
 *   g_q = (t_q I + K)^{-1} G' by one more msMINRES run, G' = G (invsqrt) or K G (sqrt),
 *   dB  = sum_q w_q g_q,
 *   dL/dK = -1/2 sum_q w_q (g_q a_q^T + a_q g_q^T)   [+ 1/2 (G A^T + A G^T) for sqrt],
 * contracted on the fly with dK/dtheta (no N x N matrix is formed):
 *   dlengthscale[n_lengthscale], doutputscale (d/d o^2), dnoise (d/d sigma^2).
 *   g: device n x s (ldg >= s); db: device n x s (lddb >= s) or NULL;
 *   each host gradient pointer may be NULL (then that contraction is skipped).
 * Synchronous. Errors as for ciq_invsqrt_mvm.
 */
int ciq_backward(const ciq_problem* p, const ciq_opts* o, int mode, const double* t,
                 const double* w, const void* solves, const void* g, int s, int ldg,
                 void* db, int lddb, double* dlengthscale, double* doutputscale,
                 double* dnoise, ciq_info* info, hipStream_t stream);

/*
 * K_p^{-1/2} B_p for nprob independent problems of uneven n_p and d_p in one
 * run: every iteration launches ONE persistent kernel-product kernel (a grid
 * of the blocks the device holds at once, taking (problem, row block, column
 * range) items from a global counter, largest problem first, skipping
 * problems that have stopped), then the inner-product, scalar and update
 * kernels; with opts->graph the iteration's kernels are replayed from a HIP
 * graph. The products stream one resident FP32 matrix per problem (FP64
 * entries rounded once; ciq_opts.kernel_cache) or evaluate FP32 entries on
 * the fly. Row tiles and column ranges per item are picked by the autotuner
 * (see ciq_opts.kernel_cache's neighbours: the tuning cache file is
 * $CIQ_TUNE_CACHE, else $HOME/.cache/libciq/tune.txt; empty disables it).
 * Each problem has its own eigenvalue bounds, shifts, Lanczos and Givens
 * state and stops on its own. All problems share kernel type, dtype
 * (CIQ_F32), s, q.
 *   probs: host array [nprob]; b, out: host arrays [nprob] of device pointers
 *   (n_p x s, contiguous); infos: host array [nprob].
 * Synchronous. Errors as for ciq_invsqrt_mvm.
 */
int ciq_invsqrt_mvm_batched(int nprob, const ciq_problem* probs, const ciq_opts* o,
                            const void* const* b, int s, void* const* out,
                            ciq_info* infos, hipStream_t stream);

/*
 * Rank-`rank` partial pivoted Cholesky factor of the noise-free kernel matrix
 * Ktil = outputscale * k(X, X), the preconditioner factor of Appendix D
 * (greedy rule of Harbrecht, Peters and Schneider 2012): step m takes the row p
 * with the largest residual diagonal d_p (ties: the smaller row), sets
 *   Lbar[i][m] = (Ktil[i][p] - sum_{k<m} Lbar[i][k] Lbar[p][k]) / sqrt(d_p)
 * for rows not yet chosen (sqrt(d_p) at p, 0 at earlier pivots) and lowers
 * d_i by Lbar[i][m]^2. It stops early once the largest residual diagonal is
 * <= 1e-10 * outputscale (numerical rank reached); later columns are 0.
 * Entries and sums in FP64 from the points converted to FP64.
 *   dtype: element type of X (CIQ_F64: double; any other dtype: float).
 *   l_out: device, n x rank doubles, row-major (ld = rank), overwritten.
 *   piv_out: host, rank ints, the row chosen at each step (-1 after a stop).
 *   trace_out: host, nullable: trace of Ktil - Lbar Lbar^T at the end.
 * Synchronous. Errors: CIQ_EINVAL (problem, dtype, pointers, rank < 1 or
 * rank > min(n, CIQ_MAX_RANK)), CIQ_ENOMEM, CIQ_EHIP.
 */
int ciq_pivoted_cholesky(const ciq_problem* p, int dtype, int rank, double* l_out,
                         int* piv_out, double* trace_out, hipStream_t stream);

/*
 * msMINRES-CIQ with a caller's sparse symmetric positive-definite operator A
 * in place of the kernel matrix (the structured operators of Sec. 5.3, e.g.
 * the precision g_obs A^T A + g_prior L of an image model, whose Gibbs
 * sampler draws mean + A^{-1/2} eps): out = A^{-1/2} B (mode CIQ_INVSQRT) or
 * A^{1/2} B (CIQ_SQRT). Products are one FP64 CSR product per iteration
 * (entries of each row in storage order); everything else as for
 * ciq_invsqrt_mvm. Without given bounds the Lanczos estimate uses
 * lambda_min = theta_min / 2 (no known floor). Symmetry and definiteness are
 * the caller's (not checked; a violation shows as non-convergence or
 * CIQ_ENUMERIC).
 *   a: host struct of device arrays; b, out: device n x s doubles.
 * Before any product the arrays' structure is checked on the device
 * (row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz, every col_idx in
 * [0, n)); a malformed operator is CIQ_EINVAL. row_ptr must hold n + 1 and
 * col_idx / val nnz entries (not checkable).
 * Synchronous. Errors: CIQ_EINVAL (a, its arrays, n, mode, a malformed CSR
 * structure, and the checks of ciq_invsqrt_mvm); CIQ_ENOTSUP unless
 * o->dtype == CIQ_F64 and o->precond_rank == 0.
 */
int ciq_csr_mvm(const ciq_csr* a, int mode, const ciq_opts* o, const double* b, int s, int ldb,
                double* out, int ldo, ciq_info* info, hipStream_t stream);

/*
 * CIQ-whitened SVGP predictive distribution in natural parameters (Sec. 5.1,
 * App. E). Inducing points Z (z->x, M = z->n; z->noise is the jitter of
 * Kzz), test points x (nb of them), whitened variational distribution
 * q(u') = N(m', S') given by its natural parameters theta = S'^{-1} m'
 * (device, M) and Theta = -S'^{-1}/2 (device, M x M row-major, symmetric
 * negative definite). Computes
 *   a_x   = Kzz^{-1/2} k_Zx            (msMINRES-CIQ, o->dtype CIQ_F64/CIQ_F32)
 *   c_x   = (-2 Theta)^{-1} a_x        (MINRES on the dense FP64 operator -2 Theta,
 *                                       solve_max_iter / solve_tol, FP64 MFMA products)
 *   mean[b] = theta . c_b,  var[b] = k(x_b, x_b) - a_b . a_b + a_b . c_b,
 * i.e. the App. E quantities from which the O(M^2) natural-gradient step is
 * assembled (d mean / d eta = a, d var / d eta = -2 mean a, d var / d H = a a^T).
 *   x: device, nb x z->d, element type of z->x (double for CIQ_F64, else float).
 *   mean, var: device, nb doubles; a_out: device M x nb doubles or NULL.
 *   info: the CIQ run's report; info_solve: the dense solve's (nullable).
 * Synchronous. Errors: CIQ_EINVAL (problem, pointers, nb < 1, solve_max_iter < 1,
 * solve_tol < 0, and the option checks of ciq_invsqrt_mvm); CIQ_ENOTSUP for the
 * split dtypes or o->precond_rank != 0.
 */
int ciq_svgp_predict(const ciq_problem* z, const void* x, int nb, const double* theta,
                     const double* Theta, const ciq_opts* o, int solve_max_iter, double solve_tol,
                     double* mean, double* var, double* a_out, ciq_info* info,
                     ciq_info* info_solve, hipStream_t stream);

/*
 * One natural-gradient step of the whitened SVGP in natural parameters
 * (App. E, the O(M^2) update): with a_b = Kzz^{-1/2} k_Zx_b and mean_b for a
 * minibatch of nb points (the a_out and mean of ciq_svgp_predict) and the
 * likelihood's constants c_mean_b = d ELL_b / d mean_b, c_var_b = d ELL_b / d var_b
 * (Gaussian likelihood: (y_b - mean_b) / noise and -1 / (2 noise)), the
 * ELBO gradient in the expectation parameters is
 *   d ELBO / d eta = scale sum_b (c_mean_b - 2 c_var_b mean_b) a_b - theta,
 *   d ELBO / d H   = scale sum_b c_var_b a_b a_b^T - I/2 - Theta
 * (scale = N / nb for a minibatch of N data; the KL derivatives are theta and
 * I/2 + Theta), and the step ascends the ELBO:
 *   theta += step * d ELBO / d eta,   Theta += step * d ELBO / d H.
 * The rank-nb update of Theta runs on FP64 MFMA (2 M^2 nb flops).
 *   a: device M x nb doubles (row-major); mean, c_mean, c_var: device nb doubles;
 *   theta: device M doubles, Theta: device M x M doubles (row-major), both
 *   updated in place.
 * Synchronous. Errors: CIQ_EINVAL (M < 1, nb < 1, null pointers, non-finite
 * scale or step), CIQ_ENOMEM, CIQ_EHIP.
 */
int ciq_svgp_ngd_step(int M, int nb, const double* a, const double* mean, const double* c_mean,
                      const double* c_var, double scale, double step, double* theta, double* Theta,
                      hipStream_t stream);

/*
 * Posterior covariance root for Thompson sampling (Sec. 5.2): with candidates
 * X* (cand->x, T = cand->n points) and observations X (x_obs, n_obs points)
 * under the same kernel,
 *   Sigma = o^2 k(X*, X*) + jitter I
 *           - o^2 k(X*, X) (o^2 k(X, X) + obs_noise I)^{-1} o^2 k(X, X*),
 * jitter = cand->noise, and out = Sigma^{1/2} B (mode CIQ_SQRT; a posterior
 * sample is mean + Sigma^{1/2} eps) or Sigma^{-1/2} B (CIQ_INVSQRT) by
 * msMINRES-CIQ exactly as ciq_sqrt_mvm / ciq_invsqrt_mvm do for K. Every
 * product with Sigma is the candidate kernel product (on the fly or resident,
 * any dtype) plus the FP64 low-rank correction -W (W^T v), W = Ksx L^{-T}
 * with L L^T = Kxx + obs_noise I factored once per call on the device
 * (blocked Cholesky and triangular solve on FP64 MFMA; n_obs <= CIQ_MAX_OBS;
 * the correction costs O(T n_obs s) per product). The
 * eigenvalue floor is the jitter (Sigma - jitter I is a covariance).
 *   x_obs: device, n_obs x cand->d, same element type as cand->x.
 *   b, out, s, ldb, ldo, o, info: as for ciq_sqrt_mvm (no per-shift solves).
 * Synchronous. Errors: those of ciq_sqrt_mvm; CIQ_EINVAL also for x_obs NULL,
 * n_obs out of [1, CIQ_MAX_OBS], obs_noise < 0 or a bad mode; CIQ_ENUMERIC if
 * Kxx + obs_noise I is not numerically positive definite; CIQ_ENOTSUP with
 * o->precond_rank != 0.
 */
int ciq_posterior_mvm(const ciq_problem* cand, const void* x_obs, int n_obs, double obs_noise,
                      int mode, const ciq_opts* o, const void* b, int s, int ldb, void* out,
                      int ldo, ciq_info* info, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CIQ_H */
