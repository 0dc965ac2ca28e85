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
// diagonal matrix, written without cancellation). Everything here is FP64:
// the two contractions of an application (U^T x, then U T) on FP64 MFMA,
// O(n R s) per application, small next to the O(n^2 s) kernel product it
// accompanies; the factorisation is O(n R^2) VALU work once per call.
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
// Both are dense FP64 contractions and run on v_mfma_f64_16x16x4_f64: lane l
// supplies A-operand element [l%16][l/16] and B-operand element [l/16][l%16];
// the accumulator holds D[l/16 + 4v][l%16] in register v.
typedef double pdx4 __attribute__((ext_vector_type(4)));

// part: the block owns 128 r x 64 s of one row chunk; wave w the r-tiles
// r0 + 32 w + {0, 16} against four 16-column s-tiles (8 accumulators).
// MFMA (i, k, j) = (r, row, s): A-operand A[row][r] (16 consecutive r per
// row, loaded into registers one group of four k-steps ahead), B-operand
// X[row][s] from double-buffered LDS tiles of 16 rows shared by the four
// waves (X is read once per block instead of once per wave).
constexpr int kPartRows = 16;
__global__ __launch_bounds__(256) void lr_part_kernel(const double* __restrict__ A, int lda,
                                                      const double* __restrict__ X, int ldx, int n, int R, int S,
                                                      int rows_per_chunk, double* __restrict__ part,
                                                      const int* done) {
    if (done != nullptr && *done) return;
    __shared__ double Xs[2][kPartRows][80];
    const int chunk = blockIdx.x, tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int r0 = blockIdx.y * 128 + wave * 32, s0 = blockIdx.z * 64;
    const int i0 = chunk * rows_per_chunk;
    const int i1 = min(n, i0 + rows_per_chunk);
    const bool ra_ok[2] = {r0 + lr < R, r0 + 16 + lr < R};
    pdx4 acc[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) acc[t][sb] = pdx4{0.0, 0.0, 0.0, 0.0};
    double ga[4][2], xn[4];
    auto load_a = [&](int ib, double (&dst)[4][2]) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int i = ib + 4 * g + lk;
            const bool iok = i < i1;
            const double* ar = A + (long long)i * lda + r0 + lr;
#pragma unroll
            for (int t = 0; t < 2; ++t) dst[g][t] = (iok && ra_ok[t]) ? ar[16 * t] : 0.0;
        }
    };
    auto load_x = [&](int ib) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = tid + 256 * k, row = e >> 6, cc = e & 63;
            const int i = ib + row, c = s0 + cc;
            xn[k] = (i < i1 && c < S) ? X[(long long)i * ldx + c] : 0.0;
        }
    };
    auto store_x = [&](int buf) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = tid + 256 * k;
            Xs[buf][e >> 6][e & 63] = xn[k];
        }
    };
    if (i0 < i1) {
        load_x(i0);
        store_x(0);
        load_a(i0, ga);
    }
    __syncthreads();
    int cur = 0;
    for (int ib = i0; ib < i1; ib += kPartRows) {
        const bool more = ib + kPartRows < i1;
        double gn[4][2];
        if (more) {
            load_x(ib + kPartRows);
            load_a(ib + kPartRows, gn);
        }
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int sb = 0; sb < 4; ++sb)
                    acc[t][sb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[g][t], Xs[cur][4 * g + lk][sb * 16 + lr],
                                                                      acc[t][sb], 0, 0, 0);
        if (more) {
            store_x(cur ^ 1);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                ga[g][0] = gn[g][0];
                ga[g][1] = gn[g][1];
            }
        }
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            const int sc = s0 + sb * 16 + lr;
            if (sc >= S) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + 16 * t + lk + 4 * v;
                if (r < R) part[((long long)chunk * R + r) * S + sc] = acc[t][sb][v];
            }
        }
}

// T[r][c] = f_r sum_ch part[ch][r][c]: 16 elements x 16 lanes per block; lane
// g sums chunks g, g + 16, ... (independent loads in flight), then the 16
// lane sums are added in lane order (deterministic).
__global__ __launch_bounds__(256) void lr_reduce_kernel(const double* __restrict__ part, int nchunk, int R, int S,
                                                        const double* __restrict__ f, double* __restrict__ T, int ldt,
                                                        const int* done) {
    if (done != nullptr && *done) return;
    __shared__ double red[16][17];
    const int el = threadIdx.x & 15, g = threadIdx.x >> 4;
    const long long total = (long long)R * S;
    const long long e = (long long)blockIdx.x * 16 + el;
    double acc = 0.0;
    if (e < total) {
#pragma unroll 4
        for (int ch = g; ch < nchunk; ch += 16) acc += part[(long long)ch * total + e];
    }
    red[g][el] = acc;
    __syncthreads();
    if (threadIdx.x < 16 && e < total) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) sum += red[k][el];
        const int r = (int)(e / S), c = (int)(e - (long long)r * S);
        if (f != nullptr) sum *= f[r];
        T[(long long)r * ldt + c] = sum;
    }
}

// apply: the block owns 64 rows x 64 s; wave w rows i0 + 16 w against four
// s-tiles. MFMA (i, k, j) = (row, r, s): A-operand A[row][r] (each lane walks
// its row, loaded into registers one slab ahead), B-operand T[r][s] from
// double-buffered LDS slabs of 32 r shared by the four waves (T is read once
// per block instead of once per wave). The slabs (36 KB) are the block's
// only LDS -- the column-sum scratch reuses them after the last slab -- so
// four blocks fit on a CU and a 50,000-row launch (782 blocks) is resident
// at once.
constexpr int kApplySlab = 32;
constexpr int kApplyLd = 72;
__global__ __launch_bounds__(256) void lr_apply_kernel(double alpha0, const double* X, int ldx,
                                                       const double* __restrict__ A, int lda,
                                                       const double* __restrict__ T, int ldt, int n, int R, int S,
                                                       double* Y, int ldy, double* __restrict__ dotp,
                                                       const int* __restrict__ colmask, const int* done,
                                                       int accumulate) {
    if (done != nullptr && *done) return;
    __shared__ double lds[2 * kApplySlab * kApplyLd];
    static_assert(16 * 64 <= 2 * kApplySlab * kApplyLd, "column-sum scratch must fit in the slab buffers");
    auto Ts = reinterpret_cast<double (*)[kApplySlab][kApplyLd]>(lds);
    auto red = reinterpret_cast<double (*)[64]>(lds);   // after the slab loop only
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int i0 = blockIdx.x * 64, s0 = blockIdx.y * 64;
    const int ia = i0 + wave * 16 + lr;           // this lane's A-operand row
    const bool ia_ok = ia < n;
    const double* arow = A + (long long)(ia_ok ? ia : 0) * lda;
    pdx4 acc[4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) acc[sb] = pdx4{0.0, 0.0, 0.0, 0.0};
    constexpr int G = kApplySlab / 4;             // k-steps per slab
    double ga[G], tn[8];
    auto load_a = [&](int rb, double* dst) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int r = rb + 4 * g + lk;
            dst[g] = (ia_ok && r < R) ? arow[r] : 0.0;
        }
    };
    auto load_t = [&](int rb) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = tid + 256 * k, rr = e >> 6, cc = e & 63;
            const int r = rb + rr, c = s0 + cc;
            tn[k] = (r < R && c < S) ? T[(long long)r * ldt + c] : 0.0;
        }
    };
    auto store_t = [&](int buf) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = tid + 256 * k;
            Ts[buf][e >> 6][e & 63] = tn[k];
        }
    };
    const int nslab = (R + kApplySlab - 1) / kApplySlab;
    load_t(0);
    store_t(0);
    load_a(0, ga);
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        const int cur = sl & 1;
        double gn[G];
        const bool more = sl + 1 < nslab;
        if (more) {
            load_t((sl + 1) * kApplySlab);
            load_a((sl + 1) * kApplySlab, gn);
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int sb = 0; sb < 4; ++sb)
                acc[sb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[g], Ts[cur][4 * g + lk][sb * 16 + lr], acc[sb], 0,
                                                               0, 0);
        if (more) {
            store_t(cur ^ 1);
#pragma unroll
            for (int g = 0; g < G; ++g) ga[g] = gn[g];
        }
        __syncthreads();
    }
    double dsum[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
        const int c = s0 + sb * 16 + lr;
        if (c >= S) continue;
        if (colmask != nullptr && colmask[c] == 0) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + wave * 16 + lk + 4 * v;
            if (i >= n) continue;
            const double x = (X != nullptr) ? X[(long long)i * ldx + c] : 0.0;
            double y = alpha0 * x + acc[sb][v];
            if (accumulate) y += Y[(long long)i * ldy + c];
            Y[(long long)i * ldy + c] = y;
            dsum[sb] = fma(x, y, dsum[sb]);
        }
    }
    if (dotp == nullptr) return;
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) red[wave * 4 + lk][sb * 16 + lr] = dsum[sb];
    __syncthreads();
    if (tid < 64 && s0 + tid < S) {
        double sum = 0.0;
#pragma unroll
        for (int g = 0; g < 16; ++g) sum += red[g][tid];
        dotp[(long long)blockIdx.x * S + s0 + tid] = sum;
    }
}

// out[c] = sum_b dotp[b][c]: 64 columns x 16 lanes per block, lane g sums
// blocks g, g + 16, ..., then the lane sums in lane order.
__global__ __launch_bounds__(1024) void lr_dotsum_kernel(const double* __restrict__ dotp, int nblk, int S,
                                                         double* __restrict__ out, const int* done) {
    if (done != nullptr && *done) return;
    __shared__ double red[16][64];
    const int cl = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl;
    double acc = 0.0;
    if (c < S) {
#pragma unroll 4
        for (int b = g; b < nblk; b += 16) acc += dotp[(long long)b * S + c];
    }
    red[g][cl] = acc;
    __syncthreads();
    if (g == 0 && c < S) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) sum += red[k][cl];
        out[c] = sum;
    }
}

struct XScale {
    double v[CIQ_MAX_D];
};

// Cross-kernel matrix out[i][j] = o2 k(xa_i, xb_j) (FP64; raw coordinates,
// per-dimension scales on the differences as in every product). One thread
// per entry, j fastest (coalesced writes).
template <int KERNEL, bool ARD>
__global__ __launch_bounds__(256) void xkernel_kernel(const double* __restrict__ xa, int na,
                                                      const double* __restrict__ xb, int nb, int dp, XScale sc,
                                                      double o2, double* __restrict__ out, int ldo) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)na * nb) return;
    const int i = (int)(e / nb), j = (int)(e - (long long)i * nb);
    double r2 = 0.0;
    for (int k = 0; k < dp; ++k) {
        const double dd = xa[(long long)i * dp + k] - xb[(long long)j * dp + k];
        if constexpr (ARD) {
            const double u = dd * sc.v[k];
            r2 = fma(u, u, r2);
        } else {
            r2 = fma(dd, dd, r2);
        }
    }
    if constexpr (!ARD) r2 *= sc.v[0] * sc.v[0];
    out[(long long)i * ldo + j] = o2 * mfma::kentry64<KERNEL>(r2);
}

// y = alpha x (n doubles).
__global__ void scale_kernel(const double* __restrict__ x, double alpha, double* __restrict__ y, long long n) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e < n) y[e] = alpha * x[e];
}

// Per column b of the M x nb arrays a, c (row-major): mean[b] = theta . c_b,
// var[b] = kxx - a_b . a_b + a_b . c_b; one block per column, fixed-order
// tree reduction.
__global__ __launch_bounds__(256) void svgp_stats_kernel(const double* __restrict__ a, const double* __restrict__ c,
                                                         const double* __restrict__ theta, int M, int nb, double kxx,
                                                         double* __restrict__ mean, double* __restrict__ var) {
    __shared__ double s1[256], s2[256], s3[256];
    const int b = blockIdx.x, t = threadIdx.x;
    double aa = 0.0, ac = 0.0, tc = 0.0;
    for (int i = t; i < M; i += 256) {
        const double av = a[(long long)i * nb + b], cv = c[(long long)i * nb + b];
        aa = fma(av, av, aa);
        ac = fma(av, cv, ac);
        tc = fma(theta[i], cv, tc);
    }
    s1[t] = aa;
    s2[t] = ac;
    s3[t] = tc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            s1[t] += s1[t + w];
            s2[t] += s2[t + w];
            s3[t] += s3[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        mean[b] = s3[0];
        var[b] = kxx - s1[0] + s2[0];
    }
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

// Row chunks per (r, s) tile: at most 1024 blocks in all (four per CU), so
// that no CU holds a fifth block that would set the launch's duration.
int lr_part_chunks(int n, int R, int S) {
    const int tiles = ((R + 127) / 128) * ((S + 63) / 64);
    int nchunk = 1024 / tiles;
    nchunk = std::min(nchunk, (n + 63) / 64);
    return std::max(nchunk, 1);
}

hipError_t launch_lr_part(const double* A, int lda, const double* X, int ldx, int n, int R, int S, int nchunk,
                          double* part, const int* done, hipStream_t st) {
    const int rows_per_chunk = (n + nchunk - 1) / nchunk;
    dim3 grid(nchunk, (R + 127) / 128, (S + 63) / 64);
    hipLaunchKernelGGL(lr_part_kernel, grid, dim3(256), 0, st, A, lda, X, ldx, n, R, S, rows_per_chunk, part,
                       done);
    return hipGetLastError();
}

hipError_t launch_lr_reduce(const double* part, int nchunk, int R, int S, const double* f, double* T, int ldt,
                            const int* done, hipStream_t st) {
    const long long total = (long long)R * S;
    hipLaunchKernelGGL(lr_reduce_kernel, dim3((unsigned)((total + 15) / 16)), dim3(256), 0, st, part, nchunk, R,
                       S, f, T, ldt, done);
    return hipGetLastError();
}

int lr_apply_blocks(int n) { return (n + 63) / 64; }

hipError_t launch_lr_apply(double alpha0, const double* X, int ldx, const double* A, int lda, const double* T,
                           int ldt, int n, int R, int S, double* Y, int ldy, double* dotp, const int* colmask,
                           const int* done, hipStream_t st, int accumulate) {
    dim3 grid(lr_apply_blocks(n), (S + 63) / 64);
    hipLaunchKernelGGL(lr_apply_kernel, grid, dim3(256), 0, st, alpha0, X, ldx, A, lda, T, ldt, n, R, S, Y, ldy,
                       dotp, colmask, done, accumulate);
    return hipGetLastError();
}

hipError_t launch_lr_dotsum(const double* dotp, int nblk, int S, double* out, const int* done, hipStream_t st) {
    hipLaunchKernelGGL(lr_dotsum_kernel, dim3((S + 63) / 64), dim3(1024), 0, st, dotp, nblk, S, out, done);
    return hipGetLastError();
}

hipError_t launch_xkernel(const double* xa, int na, const double* xb, int nb, int dp, int kernel, int ard,
                          const double* scale, double o2, double* out, int ldo, hipStream_t st) {
    XScale sc;
    for (int k = 0; k < CIQ_MAX_D; ++k) sc.v[k] = scale[k];
    const long long total = (long long)na * nb;
    const dim3 g((unsigned)((total + 255) / 256)), b(256);
    if (kernel == CIQ_KERNEL_RBF) {
        if (ard) hipLaunchKernelGGL((xkernel_kernel<CIQ_KERNEL_RBF, true>), g, b, 0, st, xa, na, xb, nb, dp, sc, o2, out, ldo);
        else hipLaunchKernelGGL((xkernel_kernel<CIQ_KERNEL_RBF, false>), g, b, 0, st, xa, na, xb, nb, dp, sc, o2, out, ldo);
    } else {
        if (ard) hipLaunchKernelGGL((xkernel_kernel<CIQ_KERNEL_MATERN52, true>), g, b, 0, st, xa, na, xb, nb, dp, sc, o2, out, ldo);
        else hipLaunchKernelGGL((xkernel_kernel<CIQ_KERNEL_MATERN52, false>), g, b, 0, st, xa, na, xb, nb, dp, sc, o2, out, ldo);
    }
    return hipGetLastError();
}

hipError_t launch_scale(const double* x, double alpha, double* y, long long n, hipStream_t st) {
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, alpha, y, n);
    return hipGetLastError();
}

hipError_t launch_svgp_stats(const double* a, const double* c, const double* theta, int M, int nb, double kxx,
                             double* mean, double* var, hipStream_t st) {
    hipLaunchKernelGGL(svgp_stats_kernel, dim3(nb), dim3(256), 0, st, a, c, theta, M, nb, kxx, mean, var);
    return hipGetLastError();
}

// Natural-gradient step operands (App. E): T[b][j] = w_b a[j][b] with
// w_b = step scale c_var[b] (the rank-nb update of Theta), and
// u[b] = step scale (c_mean[b] - 2 c_var[b] mean[b]) (the update of theta).
__global__ void ngd_prep_kernel(const double* __restrict__ a, const double* __restrict__ mean,
                                const double* __restrict__ c_mean, const double* __restrict__ c_var, int M, int nb,
                                double scale, double step, double* __restrict__ T, double* __restrict__ u) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (long long)M * nb) {
        const int b = (int)(e / M), j = (int)(e - (long long)b * M);
        T[e] = step * scale * c_var[b] * a[(long long)j * nb + b];
    }
    if (e < nb) u[e] = step * scale * (c_mean[e] - 2.0 * c_var[e] * mean[e]);
}

__global__ void diag_add_kernel(double* __restrict__ A, int M, double v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) A[(long long)i * M + i] += v;
}

hipError_t launch_ngd_prep(const double* a, const double* mean, const double* c_mean, const double* c_var, int M,
                           int nb, double scale, double step, double* T, double* u, hipStream_t st) {
    const long long total = std::max((long long)M * nb, (long long)nb);
    hipLaunchKernelGGL(ngd_prep_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, mean, c_mean,
                       c_var, M, nb, scale, step, T, u);
    return hipGetLastError();
}

hipError_t launch_diag_add(double* A, int M, double v, hipStream_t st) {
    hipLaunchKernelGGL(diag_add_kernel, dim3((M + 255) / 256), dim3(256), 0, st, A, M, v);
    return hipGetLastError();
}

hipError_t launch_pc_w(const Dev& d, double* y, const double* zc, const double* zp, hipStream_t st) {
    const long long total = (long long)d.rows_total * d.s;
    hipLaunchKernelGGL(pc_w_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, d, y, zc, zp);
    return hipGetLastError();
}

}  // namespace ciq
