// Internal declarations shared by the HIP kernels (kernels.hip) and the host
// driver (host.cpp) of libciq. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "ciq.h"

namespace ciq {

// ---------------------------------------------------------------------------
// Layout of one solver run (all device memory, carved from the scratch area).
// Rows of every problem are concatenated: problem p owns rows
// [row_off[p], row_off[p] + n[p]). Every n x s block vector is row-major with
// leading dimension s ("point-major": a tile of rows is one contiguous span).
// Global column index g = p * s + c. Per-shift arrays are indexed
// [q * ncol + g]; shift tables [p * Q + q].
// ---------------------------------------------------------------------------

struct IterState {
    int iter;       // msMINRES iterations done (products with K)
    int done;       // 1 once every column stopped or iter reached the cap
    int live;       // 1 if the current iteration's scalar stage ran
    int numeric;    // 1 if a NaN/Inf Lanczos scalar was seen
};

struct ShiftCoef {          // per (shift, column), written by the scalar stage
    double delta, eps, ginv, tau, tauw;
    int upd;                // 1: this shift moves this iteration
    int pad;
};

struct Dev {
    // problem tables
    int nprob, s, Q, ncol, max_iter;
    int rows_total;         // sum of n over problems (stride of per-shift blocks)
    const int* n;           // [nprob]
    const int* row_off;     // [nprob]
    const double* t;        // [nprob * Q]
    const double* w;        // [nprob * Q]
    double tol;
    double bd_rtol;         // breakdown threshold relative to ||K q_j||
    int bounds_mode;        // 1: plain Lanczos (no shifts), record T
    // dots
    int dots_blocks;        // partial blocks per problem
    int fuse_sums;          // consumers sum the dots partials themselves, the whole
                            // block cooperating in a fixed order: bit 1 the scalar
                            // stage (both sums), bit 2 inner-product phase 1
                            // (alpha); each saves a column-sum launch
    double* dots;           // [nprob][dots_blocks][s][2] (alpha, beta^2 partials)
    double* colsum;         // [2][ncol]: block-summed alpha, beta^2
    // column state
    double* beta1;          // ||b_g||
    double* beta_cur;       // beta_j  (couples q_{j-1}, q_j)
    double* alpha;          // alpha_j of the current iteration
    double* beta_next;      // beta_{j+1}
    double* inv_beta_next;  // 1 / beta_{j+1} (0 if the column stops)
    double* beta_used;      // beta_j used in the current update
    int* colflag;           // 0 idle, 1 update shifts only, 2 update + next Lanczos vector
    int* colactive;         // column still iterating
    int* col_iters;         // iterations per column
    int* prob_done;         // [nprob]
    double* T;              // bounds mode: [max_iter][ncol][2] (alpha, beta_next)
    // shift state [Q * ncol]
    double *c1, *s1, *c2, *s2, *phibar, *relres;
    int* frozen;
    ShiftCoef* coef;
    IterState* st;
    // resident Krylov basis (nullptr: the direction recurrence): the scalar
    // stage logs each iteration's direction coefficients, the update stores
    // q_{j+1} in slot j instead of moving the per-shift directions, and the
    // combination sum_j c_j q_j is formed once after the run
    double* clog;           // [max_iter][Q * ncol][4]: delta, eps, ginv, tauw
    double* const* basis;   // [basis_slots] slot pointers, rows_total * s doubles each: slot k holds q_{k+1}
    int basis_slots;
};

// Tiled split-FP16 copy of an FP64 block vector (rows x s, point-major), the
// B operand of v_mfma_f32_16x16x32_f16: element (i, c), multiplied by a power
// of two `scale`, is stored as hi = fp16(x) and lo = fp16((x - hi) 2^11). For
// the k-step ks = i / 32 and the column block sb = c / 16 the buffer holds 64
// lanes x 8 halfs of hi (1 KB), then the same of lo; lane (c % 16) +
// 16 ((i % 32) / 8), half i % 8, so lane l of one 16-byte load holds
// B[k = 8 (l / 16) + v][c = l % 16] of that step. `nsbt` column blocks per
// k-step; rows up to the padded width of the resident matrix, zero beyond n.
__host__ __device__ inline size_t op16_index(int i, int c, int nsbt) {
    const int ks = i >> 5, r = i & 31;
    const int lane = (c & 15) + 16 * (r >> 3);
    return ((((size_t)ks * nsbt + (c >> 4)) * 2) * 64 + lane) * 8 + (r & 7);
}
inline size_t op16_halfs(size_t rows_pad, int nsbt) { return rows_pad * (size_t)nsbt * 32; }
constexpr float kOp16Scale = 256.0f;   // scale of unit-norm Lanczos vectors (entries <= 1)

// Where the update / start kernels write the split FP16 copy of the next
// product operand (p == nullptr: none).
struct Op16 {
    void* p;
    int nsbt;
    float scale;
};
// column blocks of 16 in a split operand buffer for s columns: 1, 2, 4 or a
// multiple of 8, so every launch's column blocks lie inside it
inline int op16_nsbt(int s) {
    const int nb = (s + 15) / 16;
    return nb <= 1 ? 1 : nb <= 2 ? 2 : nb <= 4 ? 4 : (nb + 7) / 8 * 8;
}

// Work list entry of the kernel-product kernel: (problem, row block).
struct WorkItem {
    int prob;
    int rb;
};

// Arguments of one kernel-product launch Y = K V (split over the j range).
struct MvmArgs {
    const void* xh;          // zero-padded FP64 points: rows x dp (FP64 path: pre-scaled;
                             // FP32 path: raw coordinates, scaled after subtraction)
    const void* v;           // rows x s (ld = ldv); float (FP32 path) or double
    void* y;                 // double partial outputs: nsplit x rows x s (ld = ldy)
    float* y32;              // set: the resident FP32 / split-FP16 products write their
                             // partials here instead, rounded once to FP32 (same layout)
    long long ysplit;        // elements between split partials
    int ldv, ldy;
    int s;
    int kernel;
    int dp;
    int nsplit;
    int rt;                  // FP32 product: row tiles of 16 per wave (1 or 2)
    int acc;                 // FP32 resident product: 1 = the finer FP64 accumulation
                             // (inverse root), 0 = the faster one (see mvm_cache.hip)
    int ard;                 // FP32 product: per-dimension scales differ
    double scale[CIQ_MAX_D]; // FP32 product: per-dimension scale of coordinate differences
    const double* pscale;    // batched: [nprob][CIQ_MAX_D] scales
    // single problem (wl == nullptr)
    int n;
    double o2, s2;
    // batched
    const WorkItem* wl;      // [nrb_total]
    int nrb;                 // number of row blocks (grid.x)
    const int* pn;           // [nprob] n per problem
    const int* poff;         // [nprob] row offset
    const float* po2;        // [nprob]
    const float* ps2;        // [nprob]
    const int* prob_done;    // [nprob] or nullptr
    const int* done;         // global done flag or nullptr
    int* queue;              // batched FP32 products: persistent work counter (nullptr: one block per item)
    int nitems;              // work items = nrb * nsplit
    const long long* pkt;    // batched resident FP32: per-problem element offset of its matrix in kt
    const long long* pnjs;   // per-problem padded columns / 4
    // resident kernel matrix (single problem): operand-tiled unit-scale
    // entries, double (CIQ_F64) or float (CIQ_F32), see mvm_cache.hip;
    // nullptr = evaluate entries on the fly
    const void* kt;
    long long njs;           // padded columns / 4
    // split FP16 resident matrix (CIQ_F16X3): the operand is the tiled split
    // copy `vt` of the FP64 vector `v` (which supplies the noise term);
    // y = o2 (K vt) * vinv (per column vcol_inv[c] when non-null)
    const void* vt;
    int nsbt;
    double vinv;
    const double* vcol_inv;
};

// Build pass of the resident kernel matrix (mvm_cache.hip).
struct KBuildArgs {
    const double* xh;        // n x dp FP64 points (raw coordinates)
    double scale[CIQ_MAX_D]; // per-dimension scale of coordinate differences
    int n, dp, kernel, ard;
    int nchunk;              // padded columns / 64
    long long njs;           // padded columns / 4
    int elem;                // 0: FP64, 1: FP32 (entries evaluated in FP64, rounded
                             // once), 2: split FP16 hi + 2^-11 lo (4 bytes per entry)
    void* kt;                // kcache_rows(n) x kcache_cols(n) entries
};
size_t kcache_rows(int n);
size_t kcache_cols(int n);
size_t kcache_bytes(int n, int elem_bytes);
hipError_t launch_kbuild(const KBuildArgs& a, hipStream_t st);
hipError_t launch_mvm_kt(const MvmArgs& a, int nsb, hipStream_t st);
hipError_t launch_mvm_kt32(const MvmArgs& a, int nsb, hipStream_t st);
hipError_t launch_mvm_kt16(const MvmArgs& a, int nsb, hipStream_t st);
// Blocks of the resident product (FP32 or FP64 operands, nsb column blocks of
// 16, rt row tiles per wave) that one CU holds at once; 0 if the query fails.
int kt_blocks_per_cu(int dtype, int nsb, int rt, int acc = 0);
// column blocks one product launch covers: 8 x 16 for the on-the-fly FP32
// product and the resident split FP16 one, 4 x 16 otherwise
inline int product_cap(int dtype, bool cached) {
    return ((dtype == CIQ_F32 && !cached) || (dtype == CIQ_F16X3 && cached)) ? 128 : 64;
}

// ---- launchers (kernels.hip, mvm_f32_*.hip) ---------------------------------
hipError_t launch_mvm_f32_rbf_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st);
hipError_t launch_mvm_f32_rbf_ard(const MvmArgs& a, int nsb, int grid_x, hipStream_t st);
hipError_t launch_mvm_f32_m52_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st);
hipError_t launch_mvm_f32_m52_ard(const MvmArgs& a, int nsb, int grid_x, hipStream_t st);
hipError_t launch_mvm_f64_rbf_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st);
hipError_t launch_mvm_f64_rbf_ard(const MvmArgs& a, int nsb, int grid_x, hipStream_t st);
hipError_t launch_mvm_f64_m52_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st);
hipError_t launch_mvm_f64_m52_ard(const MvmArgs& a, int nsb, int grid_x, hipStream_t st);
hipError_t launch_mvm_x3_rbf(const MvmArgs& a, int nsb, int grid_x, bool half, hipStream_t st);
hipError_t launch_mvm_x3_m52(const MvmArgs& a, int nsb, int grid_x, bool half, hipStream_t st);
int mvm_rows_per_block(int dtype, int s, int rt);
int mvm_pick_nsplit(int dtype, int nrb, int n_max, int s);
hipError_t launch_mvm(int dtype, const MvmArgs& a, hipStream_t st);

template <typename TI>
hipError_t launch_prep(const TI* x, int n, int d, int dp, const double* scale, double* xh,
                       hipStream_t st);

// ypart: double partials of the kernel product (both paths accumulate in FP64)
template <typename TO>
hipError_t launch_reduce_splits(const double* ypart, long long ysplit, int nsplit, int ldy,
                                int n, int s, TO* out, int ldo, hipStream_t st);

// Block partials of the inner products (phase 0: q_j^T (y - beta_j q_{j-1}),
// reducing the nsplit product partials into y's first slot; phase 1:
// ||y - beta_j q_{j-1} - alpha_j q_j||^2). y32 set (phase 0 only): the split
// partials are FP32 there and are summed in FP64 into y's first slot.
template <typename T>
hipError_t launch_dots(const Dev& d, T* y, long long ysplit, int nsplit, const T* q,
                       const T* qp, int phase, hipStream_t st, const float* y32 = nullptr);

hipError_t launch_colsum(const Dev& d, int k, hipStream_t st);
hipError_t launch_scalar_init(const Dev& d, hipStream_t st);
hipError_t launch_scalar(const Dev& d, hipStream_t st);

// q32 (nullable): FP32 copy of the next Lanczos vector, the FP32 product's operand
// pnext (nullable): preconditioned form. Then y holds the finished direction
// w (not the product), the direction recurrence consumes qcur = p_j, a
// continuing column gets qprev <- w / beta_{j+1} (z_{j+1}) and
// pnext <- pnext / beta_{j+1} (p_{j+1} = P^{-1} z_{j+1}), and q32 copies pnext.
template <typename T>
hipError_t launch_update(const Dev& d, const T* y, long long ysplit, int nsplit, const T* qcur,
                         T* qprev, const T* m_prev, T* m_cur, T* acc, T* solves, float* q32,
                         int max_n, hipStream_t st, T* pnext = nullptr, Op16 op = Op16{nullptr, 0, 1.0f});

// pvec (nullable): preconditioned start, pvec <- pvec / beta_1 too and q32
// copies pvec instead of q.
// Slot pointer table of the resident basis for slots [first, end), from the
// bases of chunks k0 .. k0 + kBasisChunksPerLaunch - 1 (passed by value).
constexpr int kBasisChunksPerLaunch = 16;
struct BasisChunks {
    char* base[kBasisChunksPerLaunch];
};
hipError_t launch_basis_table(double** tab, int first, int end, int per_chunk, size_t stride, int k0,
                              const BasisChunks& c, hipStream_t st);

// After a run with the resident basis: acc = sum_j c_j q_j per column, the
// coefficients c_j by back-substitution of the logged direction recurrence
// of every (shift, column). cq: [iters][Q * ncol], c: [iters][ncol] doubles
// of scratch; iters = the run's iteration count.
hipError_t launch_basis_combine(const Dev& d, int iters, double* cq, double* c, double* acc, int max_n,
                                hipStream_t st);

template <typename T>
hipError_t launch_init_vectors(const Dev& d, T* q, T* qprev, T* acc, float* q32, int rows,
                               hipStream_t st, T* pvec = nullptr, Op16 op = Op16{nullptr, 0, 1.0f});

// Split FP16 operand (op16_index layout, nsbt column blocks) of the n x s FP64
// block x (ld): per-column power-of-two scales (scale, inv: device [s]).
hipError_t launch_op16_split(const double* x, int n, int s, int ld, double* scale, double* inv, void* vt,
                             int nsbt, hipStream_t st);


template <typename TI, typename TO>
hipError_t launch_copy(const TI* src, int ld_src, int n, int s, TO* dst, int ld_dst,
                       hipStream_t st);

template <typename T>
hipError_t launch_fill(T* p, size_t count, T value, hipStream_t st);

template <typename T>
hipError_t launch_splitmix(T* v, int n, uint64_t seed, int ld, hipStream_t st);

// ---- pivoted-Cholesky preconditioner (precond.hip) ---------------------------
// Partial pivoted Cholesky of Ktil = o^2 k(X, X): step m reads the pivot the
// previous pick chose, writes column m of L and updates the residual diagonal;
// the pick reduces the per-block (largest residual diagonal, smallest row)
// candidates and the residual trace.
struct PcholArgs {
    const double* xh;        // n x dp FP64 points (raw coordinates)
    double scale[CIQ_MAX_D]; // per-dimension scale of coordinate differences
    int n, dp, kernel, ard;
    double o2;               // outputscale (the diagonal of Ktil)
    double stop_abs;         // stop once the largest residual diagonal <= this
    double* L;               // n x ldl, row-major; column m written at step m
    int ldl;
    double* dres;            // [n] residual diagonal
    int* chosen;             // [n] 1 once the row was a pivot
    int* piv;                // [rank + 1] pivot of step m (-1: stopped)
    double* pval;            // [rank + 1] residual diagonal of that pivot
    double* trace;           // [rank + 1] residual trace before step m
    double* bval;            // [nblk] block candidates
    int* bidx;
    double* bsum;
    int nblk;
};
hipError_t launch_pchol_init(const PcholArgs& a, hipStream_t st);
hipError_t launch_pchol_pick(const PcholArgs& a, int m, hipStream_t st);
hipError_t launch_pchol_col(const PcholArgs& a, int m, hipStream_t st);

// Low-rank pieces of P^{-1} x and P^{1/2} x (both alpha0 x + U f(U^T x)):
//   part[c][r][s] = sum_{i in chunk c} A[i][r] X[i][s]                (lr_part)
//   T[r][s] = f_r * sum_c part[c][r][s]   (f nullable: 1)             (lr_reduce)
//   Y[i][s] = alpha0 X[i][s] + sum_r A[i][r] T[r][s]  (X nullable: 0), (lr_apply)
//     optionally dotp[blk][s] = sum over the block's rows of X[i][s] Y[i][s]
//     and, with colmask, columns whose mask is 0 left untouched (dotp 0).
// `done` (nullable): skip the launch's work once the run has stopped.
int lr_part_chunks(int n, int R, int S);
hipError_t launch_lr_part(const double* A, int lda, const double* X, int ldx, int n, int R, int S,
                          int nchunk, double* part, const int* done, hipStream_t st);
hipError_t launch_lr_reduce(const double* part, int nchunk, int R, int S, const double* f, double* T,
                            int ldt, const int* done, hipStream_t st);
int lr_apply_blocks(int n);
hipError_t launch_lr_apply(double alpha0, const double* X, int ldx, const double* A, int lda,
                           const double* T, int ldt, int n, int R, int S, double* Y, int ldy,
                           double* dotp, const int* colmask, const int* done, hipStream_t st,
                           int accumulate = 0);   // 1: Y += alpha0 X + A T
// out[c] = sum_b dotp[b][c] (fixed order), b < nblk
hipError_t launch_lr_dotsum(const double* dotp, int nblk, int S, double* out, const int* done,
                            hipStream_t st);
// out[i][j] = o2 k(xa_i, xb_j), FP64 (raw coordinates, per-dimension scales
// on the differences), out row-major with leading dimension ldo >= nb.
hipError_t launch_xkernel(const double* xa, int na, const double* xb, int nb, int dp, int kernel, int ard,
                          const double* scale, double o2, double* out, int ldo, hipStream_t st);
// ---- observation-block factors of the posterior (chol.hip) ------------------
// A (npad x npad, row-major, zero-filled outside the leading n x n): A[i][i]
// += shift for i < n, identity on the padded diagonal.
hipError_t launch_chol_prep(double* A, int n, int npad, double shift, hipStream_t st);
// In-place lower Cholesky factor of A (npad a multiple of 64; the strict
// upper part of each diagonal block is zeroed, the rest of the upper
// triangle is left unspecified); dinv[k] (64 x 64 each) = inverse of
// diagonal block k. *status |= 1 if a pivot is not positive (the caller
// zeroes it).
hipError_t launch_chol_blocked(double* A, int npad, double* dinv, int* status, hipStream_t st);
// W <- W L^{-T} in place for W rows x npad (ld npad), L and dinv from
// launch_chol_blocked.
hipError_t launch_trsm_right_lt(double* W, int rows, int npad, const double* L, const double* dinv, hipStream_t st);

// ---- sparse symmetric operator (sparse.hip) ----------------------------------
struct SparseOp {
    int n;                   // rows = columns
    const int* row_ptr;      // [n + 1]
    const int* col;          // [nnz]
    const double* val;       // [nnz]
};
// *bad |= 1 unless row_ptr[0] = 0, row_ptr is non-decreasing, row_ptr[n] = nnz
// and every col[k] lies in [0, n) (the caller zeroes *bad).
hipError_t launch_csr_check(const int* row_ptr, const int* col, int n, int nnz, int* bad, hipStream_t st);
// y = A x for s columns (x: n x s, ld ldx; y: n x s, ld ldy); `done` as above.
hipError_t launch_spmv(const SparseOp& a, const double* x, int ldx, int s, double* y, int ldy, const int* done,
                       hipStream_t st);

// y = alpha x (n doubles).
hipError_t launch_scale(const double* x, double alpha, double* y, long long n, hipStream_t st);
// SVGP predictive statistics per column b (a, c: M x nb row-major):
// mean[b] = theta . c_b, var[b] = kxx - a_b . a_b + a_b . c_b.
hipError_t launch_svgp_stats(const double* a, const double* c, const double* theta, int M, int nb, double kxx,
                             double* mean, double* var, hipStream_t st);
// Natural-gradient step operands: T (nb x M) = diag(step scale c_var) a^T,
// u (nb) = step scale (c_mean - 2 c_var mean); a is M x nb row-major.
hipError_t launch_ngd_prep(const double* a, const double* mean, const double* c_mean, const double* c_var, int M,
                           int nb, double scale, double step, double* T, double* u, hipStream_t st);
// A[i][i] += v for the M x M row-major A.
hipError_t launch_diag_add(double* A, int M, double v, hipStream_t st);
// Dense symmetric operator of a single-shift solve (SVGP: -2 Theta).
struct DenseOp {
    const double* A;         // n x n, row-major
    int n;
};

// Preconditioned Lanczos direction: y <- (y - beta_j z_prev) - alpha_j z_cur
// (alpha_j from colsum[0..ncol)), in place.
hipError_t launch_pc_w(const Dev& d, double* y, const double* zc, const double* zp, hipStream_t st);

// ---- backward tile pass (grad.hip) ------------------------------------------
int grad_rows_pad(int n);
int grad_k_pad(int k);
// U/V rows: [w_q g_q(i,:) | -G(i,:)] and [a_q(i,:) | A(i,:)], zero padded to
// grad_rows_pad(n) x grad_k_pad((Q + sqrt_mode) * s)
template <typename T>
hipError_t launch_build_uv(const double* gq, const T* aq, const T* g, int ldg, const double* w_dev, int n,
                           int Q, int s, int sqrt_mode, double* U, double* V, hipStream_t st);
// partial[block][0..dp) = sum W_ij h (u_id - u_jd)^2, [dp] = sum W_ij k, [dp+1] = sum W_ii
hipError_t launch_grad_pass(int kernel, const double* U, const double* V, int kpad, const double* pts,
                            int n, int dp, double* partial, int* nblocks, hipStream_t st);

}  // namespace ciq
