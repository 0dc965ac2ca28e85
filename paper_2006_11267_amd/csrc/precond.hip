// Pivoted-Cholesky preconditioner of msMINRES-CIQ (Sec. 3.4, Appendix D).
//
// P = Lbar Lbar^T + sigma^2 I with Lbar the rank-R partial pivoted Cholesky
// factor of the noise-free kernel matrix Ktil = o^2 k(X, X) (greedy largest
// residual diagonal, Harbrecht-Peters-Schneider 2012). With
// Lbar^T Lbar = V diag(lam) V^T and U = Lbar V (n x R) both operations the
// preconditioned run needs have the form alpha0 x + U diag(f) U^T x:
//     P^{-1} x  : alpha0 = 1/sigma^2, f = -1 / (sigma^2 (lam + sigma^2))
//     P^{1/2} x : alpha0 = sigma,     f = 1 / (sqrt(lam + sigma^2) + sigma)
// (matrix inversion lemma and the exact square root of a low-rank-plus-
// diagonal matrix, written without cancellation). Everything here is FP64
// VALU work of O(n R s) per application, small next to the O(n^2 s) kernel
// product it accompanies; the factorisation is O(n R^2) once per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>

#include "ciq_internal.h"
#include "mvm_mfma.h"

namespace ciq {

namespace {

// Candidate order of the pivot search: larger residual diagonal first, then
// the smaller row index (a total order, so the reduction is deterministic).
__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

// Block reduction of (value, index) by `better` and of a sum in a fixed tree
// order; thread 0 writes the block's partial.
__device__ void block_pick(double v, int i, double sum, double* bval, int* bidx, double* bsum) {
    __shared__ double sv[256], ss[256];
    __shared__ int si[256];
    const int t = threadIdx.x;
    sv[t] = v;
    si[t] = i;
    ss[t] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            if (better(sv[t + w], si[t + w], sv[t], si[t])) {
                sv[t] = sv[t + w];
                si[t] = si[t + w];
            }
            ss[t] += ss[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        bval[blockIdx.x] = sv[0];
        bidx[blockIdx.x] = si[0];
        bsum[blockIdx.x] = ss[0];
    }
}

__global__ __launch_bounds__(256) void pchol_init_kernel(PcholArgs a) {
    double bv = -DBL_MAX, sum = 0.0;
    int bi = INT_MAX;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < a.n; i += gridDim.x * 256) {
        a.dres[i] = a.o2;
        a.chosen[i] = 0;
        sum += a.o2;
        if (better(a.o2, i, bv, bi)) {
            bv = a.o2;
            bi = i;
        }
    }
    block_pick(bv, bi, sum, a.bval, a.bidx, a.bsum);
}

// Step m's pivot from the block candidates (one block).
__global__ __launch_bounds__(256) void pchol_pick_kernel(PcholArgs a, int m) {
    double bv = -DBL_MAX, sum = 0.0;
    int bi = INT_MAX;
    for (int b = threadIdx.x; b < a.nblk; b += 256) {
        sum += a.bsum[b];
        if (better(a.bval[b], a.bidx[b], bv, bi)) {
            bv = a.bval[b];
            bi = a.bidx[b];
        }
    }
    __shared__ double sv[256], ss[256];
    __shared__ int si[256];
    const int t = threadIdx.x;
    sv[t] = bv;
    si[t] = bi;
    ss[t] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            if (better(sv[t + w], si[t + w], sv[t], si[t])) {
                sv[t] = sv[t + w];
                si[t] = si[t + w];
            }
            ss[t] += ss[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        const bool stopped = (m > 0 && a.piv[m - 1] < 0);
        const bool take = !stopped && si[0] != INT_MAX && sv[0] > a.stop_abs;
        a.piv[m] = take ? si[0] : -1;
        a.pval[m] = take ? sv[0] : 0.0;
        a.trace[m] = ss[0];
    }
}

// Column m: L[i][m] = (Ktil[i][p] - sum_{k<m} L[i][k] L[p][k]) / sqrt(d_p) for
// rows not yet chosen, sqrt(d_p) at the pivot p, 0 at earlier pivots; the
// residual diagonal loses L[i][m]^2. Then this block's candidates for step m+1.
template <int KERNEL, bool ARD>
__global__ __launch_bounds__(256) void pchol_col_kernel(PcholArgs a, int m) {
    extern __shared__ double lrow[];          // L[p][0..m)
    __shared__ double xp[CIQ_MAX_D];
    const int p = a.piv[m];
    if (p < 0) return;                        // stopped: column m stays zero
    const int dp = a.dp;
    for (int k = threadIdx.x; k < m; k += 256) lrow[k] = a.L[(long long)p * a.ldl + k];
    if (threadIdx.x < dp) xp[threadIdx.x] = a.xh[(long long)p * dp + threadIdx.x];
    __syncthreads();
    const double lpp = sqrt(a.pval[m]);
    const double sc0sq = a.scale[0] * a.scale[0];
    double bv = -DBL_MAX, sum = 0.0;
    int bi = INT_MAX;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < a.n; i += gridDim.x * 256) {
        if (a.chosen[i]) continue;
        double* li = a.L + (long long)i * a.ldl;
        if (i == p) {
            li[m] = lpp;
            a.chosen[i] = 1;
            a.dres[i] = 0.0;
            continue;
        }
        double r2 = 0.0;
        for (int k = 0; k < dp; ++k) {
            const double dd = a.xh[(long long)i * dp + k] - xp[k];
            if constexpr (ARD) {
                const double u = dd * a.scale[k];
                r2 = fma(u, u, r2);
            } else {
                r2 = fma(dd, dd, r2);
            }
        }
        if constexpr (!ARD) r2 *= sc0sq;
        const double kip = a.o2 * mfma::kentry64<KERNEL>(r2);
        double s = 0.0;
        for (int k = 0; k < m; ++k) s = fma(li[k], lrow[k], s);
        const double l = (kip - s) / lpp;
        li[m] = l;
        const double di = a.dres[i] - l * l;
        a.dres[i] = di;
        sum += di;
        if (better(di, i, bv, bi)) {
            bv = di;
            bi = i;
        }
    }
    block_pick(bv, bi, sum, a.bval, a.bidx, a.bsum);
}

// ---- low-rank products -------------------------------------------------------
// Tile 32 r x 64 s per block, 32-row slabs of A and X staged in LDS; thread
// (tr, tc) accumulates r = r0 + 2 tr + {0,1}, s = s0 + tc + 16 k, k = 0..3.
__global__ __launch_bounds__(256) void lr_part_kernel(const double* __restrict__ A, int lda,
                                                      const double* __restrict__ X, int ldx, int n, int R, int S,
                                                      int rows_per_chunk, double* __restrict__ part,
                                                      const int* done) {
    if (done != nullptr && *done) return;
    __shared__ double As[32][33];
    __shared__ double Xs[32][64];
    const int chunk = blockIdx.x, r0 = blockIdx.y * 32, c0 = blockIdx.z * 64;
    const int i0 = chunk * rows_per_chunk;
    const int i1 = min(n, i0 + rows_per_chunk);
    const int t = threadIdx.x, tc = t & 15, tr = t >> 4;
    double acc[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    for (int ib = i0; ib < i1; ib += 32) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = t + 256 * k, row = e >> 5, rr = e & 31;
            const int i = ib + row, r = r0 + rr;
            As[row][rr] = (i < i1 && r < R) ? A[(long long)i * lda + r] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = t + 256 * k, row = e >> 6, cc = e & 63;
            const int i = ib + row, c = c0 + cc;
            Xs[row][cc] = (i < i1 && c < S) ? X[(long long)i * ldx + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int row = 0; row < 32; ++row) {
            const double a0 = As[row][2 * tr], a1 = As[row][2 * tr + 1];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double x = Xs[row][tc + 16 * k];
                acc[0][k] = fma(a0, x, acc[0][k]);
                acc[1][k] = fma(a1, x, acc[1][k]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int r = r0 + 2 * tr + u;
        if (r >= R) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = c0 + tc + 16 * k;
            if (c < S) part[((long long)chunk * R + r) * S + c] = acc[u][k];
        }
    }
}

__global__ void lr_reduce_kernel(const double* __restrict__ part, int nchunk, int R, int S,
                                 const double* __restrict__ f, double* __restrict__ T, int ldt, const int* done) {
    if (done != nullptr && *done) return;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)R * S;
    if (e >= total) return;
    const int r = (int)(e / S), c = (int)(e - (long long)r * S);
    double s = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) s += part[(long long)ch * total + e];
    if (f != nullptr) s *= f[r];
    T[(long long)r * ldt + c] = s;
}

// Tile 64 rows x 64 s per block, r in slabs of 32 through LDS; thread (tr, tc)
// owns rows i0 + tr + 16 u and columns s0 + tc + 16 k (u, k = 0..3).
__global__ __launch_bounds__(256) void lr_apply_kernel(double alpha0, const double* X, int ldx,
                                                       const double* __restrict__ A, int lda,
                                                       const double* __restrict__ T, int ldt, int n, int R, int S,
                                                       double* Y, int ldy, double* __restrict__ dotp,
                                                       const int* __restrict__ colmask, const int* done) {
    if (done != nullptr && *done) return;
    __shared__ double As[64][33];
    __shared__ double Ts[32][64];
    __shared__ double red[16][64];
    const int i0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    const int t = threadIdx.x, tc = t & 15, tr = t >> 4;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[u][k] = 0.0;
    for (int r0 = 0; r0 < R; r0 += 32) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = t + 256 * k, row = e >> 5, rr = e & 31;
            const int i = i0 + row, r = r0 + rr;
            As[row][rr] = (i < n && r < R) ? A[(long long)i * lda + r] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = t + 256 * k, rr = e >> 6, cc = e & 63;
            const int r = r0 + rr, c = c0 + cc;
            Ts[rr][cc] = (r < R && c < S) ? T[(long long)r * ldt + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < 32; ++rr) {
            double av[4], tv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) av[u] = As[tr + 16 * u][rr];
#pragma unroll
            for (int k = 0; k < 4; ++k) tv[k] = Ts[rr][tc + 16 * k];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[u][k] = fma(av[u], tv[k], acc[u][k]);
        }
    }
    double dsum[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = c0 + tc + 16 * k;
        if (c >= S) continue;
        if (colmask != nullptr && colmask[c] == 0) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + tr + 16 * u;
            if (i >= n) continue;
            const double x = (X != nullptr) ? X[(long long)i * ldx + c] : 0.0;
            const double y = alpha0 * x + acc[u][k];
            Y[(long long)i * ldy + c] = y;
            dsum[k] = fma(x, y, dsum[k]);
        }
    }
    if (dotp == nullptr) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) red[tr][tc + 16 * k] = dsum[k];
    __syncthreads();
    if (t < 64 && c0 + t < S) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) s += red[r][t];
        dotp[(long long)blockIdx.x * S + c0 + t] = s;
    }
}

__global__ void lr_dotsum_kernel(const double* __restrict__ dotp, int nblk, int S, double* __restrict__ out,
                                 const int* done) {
    if (done != nullptr && *done) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= S) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += dotp[(long long)b * S + c];
    out[c] = s;
}

// Single-problem runs only (the preconditioned path is not batched).
__global__ void pc_w_kernel(Dev d, double* __restrict__ y, const double* __restrict__ zc,
                            const double* __restrict__ zp) {
    if (d.st->done) return;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)d.rows_total * d.s;
    if (e >= total) return;
    const int c = (int)(e % d.s);
    if (!d.colactive[c]) return;
    const double bj = d.beta_cur[c], al = d.colsum[c];
    const double vT = y[e] - bj * zp[e];       // the order of the alpha inner product
    y[e] = vT - al * zc[e];
}

}  // namespace

hipError_t launch_pchol_init(const PcholArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(pchol_init_kernel, dim3(a.nblk), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_pchol_pick(const PcholArgs& a, int m, hipStream_t st) {
    hipLaunchKernelGGL(pchol_pick_kernel, dim3(1), dim3(256), 0, st, a, m);
    return hipGetLastError();
}

hipError_t launch_pchol_col(const PcholArgs& a, int m, hipStream_t st) {
    const size_t shm = (size_t)(m > 0 ? m : 1) * sizeof(double);
    const dim3 g(a.nblk), b(256);
    if (a.kernel == CIQ_KERNEL_RBF) {
        if (a.ard) hipLaunchKernelGGL((pchol_col_kernel<CIQ_KERNEL_RBF, true>), g, b, shm, st, a, m);
        else hipLaunchKernelGGL((pchol_col_kernel<CIQ_KERNEL_RBF, false>), g, b, shm, st, a, m);
    } else {
        if (a.ard) hipLaunchKernelGGL((pchol_col_kernel<CIQ_KERNEL_MATERN52, true>), g, b, shm, st, a, m);
        else hipLaunchKernelGGL((pchol_col_kernel<CIQ_KERNEL_MATERN52, false>), g, b, shm, st, a, m);
    }
    return hipGetLastError();
}

int lr_part_chunks(int n, int R, int S) {
    const int tiles = ((R + 31) / 32) * ((S + 63) / 64);
    int nchunk = (1024 + tiles - 1) / tiles;
    nchunk = std::min(nchunk, (n + 63) / 64);
    return std::max(nchunk, 1);
}

hipError_t launch_lr_part(const double* A, int lda, const double* X, int ldx, int n, int R, int S, int nchunk,
                          double* part, const int* done, hipStream_t st) {
    const int rows_per_chunk = (n + nchunk - 1) / nchunk;
    dim3 grid(nchunk, (R + 31) / 32, (S + 63) / 64);
    hipLaunchKernelGGL(lr_part_kernel, grid, dim3(256), 0, st, A, lda, X, ldx, n, R, S, rows_per_chunk, part,
                       done);
    return hipGetLastError();
}

hipError_t launch_lr_reduce(const double* part, int nchunk, int R, int S, const double* f, double* T, int ldt,
                            const int* done, hipStream_t st) {
    const long long total = (long long)R * S;
    hipLaunchKernelGGL(lr_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, nchunk, R,
                       S, f, T, ldt, done);
    return hipGetLastError();
}

int lr_apply_blocks(int n) { return (n + 63) / 64; }

hipError_t launch_lr_apply(double alpha0, const double* X, int ldx, const double* A, int lda, const double* T,
                           int ldt, int n, int R, int S, double* Y, int ldy, double* dotp, const int* colmask,
                           const int* done, hipStream_t st) {
    dim3 grid(lr_apply_blocks(n), (S + 63) / 64);
    hipLaunchKernelGGL(lr_apply_kernel, grid, dim3(256), 0, st, alpha0, X, ldx, A, lda, T, ldt, n, R, S, Y, ldy,
                       dotp, colmask, done);
    return hipGetLastError();
}

hipError_t launch_lr_dotsum(const double* dotp, int nblk, int S, double* out, const int* done, hipStream_t st) {
    hipLaunchKernelGGL(lr_dotsum_kernel, dim3((S + 63) / 64), dim3(64), 0, st, dotp, nblk, S, out, done);
    return hipGetLastError();
}

hipError_t launch_pc_w(const Dev& d, double* y, const double* zc, const double* zp, hipStream_t st) {
    const long long total = (long long)d.rows_total * d.s;
    hipLaunchKernelGGL(pc_w_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, d, y, zc, zp);
    return hipGetLastError();
}

}  // namespace ciq
