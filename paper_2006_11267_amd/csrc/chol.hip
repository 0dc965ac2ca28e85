// Factors of the posterior covariance's observation block (Sec. 5.2):
// Sigma = Kss + jitter I - W W^T with W = Ksx L^{-T} and L L^T = Kxx +
// sigma_obs^2 I. Right-looking blocked Cholesky in 64-column panels and the
// right-side triangular solve for W, both on FP64 MFMA.
//
// The matrix is padded to npad = 64 * ceil(n / 64) rows and columns with the
// identity on the padded diagonal and zeros elsewhere, so the factor is
// blockdiag(L, I) and every panel is a full 64 wide; zero-padded columns of
// Ksx stay zero in W. Per panel k:
//   chol_diag: one workgroup factors the 64 x 64 diagonal block in LDS and
//              writes its inverse D_k = L_kk^{-1} (forward substitution)
//   panel:     L[below, k] = A[below, k] D_k^T           (gemm_nt, in place)
//   trailing:  A[i, j] -= L[i, k] L[j, k]^T, lower tiles (gemm_nt)
// and for W, per block column k in order:
//   W[:, k] = R[:, k] D_k^T;  R[:, later] -= W[:, k] L[later, k]^T
// where R starts as Ksx and is overwritten by W.
#include <hip/hip_runtime.h>

#include "ciq_internal.h"

namespace ciq {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int CB = 64;        // panel width
constexpr int CLD = CB + 1;   // LDS row stride (doubles): rows land on different banks

// A[i][i] += shift for i < n; padded rows n..npad-1 get 1 on the diagonal
// (the caller zero-fills the padded rows and columns)
__global__ void chol_prep_kernel(double* __restrict__ A, int n, int npad, double shift) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    double* d = A + (size_t)i * npad + i;
    *d = (i < n) ? *d + shift : 1.0;
}

// Lower Cholesky factor of the diagonal block at (k0, k0) in place and its
// inverse into dinv (64 x 64 row-major). A pivot that is not positive and
// finite sets *status to 1 and is replaced by 1 so the rest stays finite.
__global__ __launch_bounds__(256) void chol_diag_kernel(double* __restrict__ A, int ld, int k0,
                                                        double* __restrict__ dinv, int* __restrict__ status) {
    __shared__ double a[CB][CLD];
    __shared__ double x[CB][CLD];
    const int tid = threadIdx.x;
    double* blk = A + (size_t)k0 * ld + k0;
    for (int e = tid; e < CB * CB; e += 256) a[e / CB][e % CB] = blk[(size_t)(e / CB) * ld + e % CB];
    __syncthreads();
    for (int j = 0; j < CB; ++j) {
        if (tid == 0) {
            double dj = a[j][j];
            if (!(dj > 0.0) || !isfinite(dj)) {
                *status = 1;
                dj = 1.0;
            }
            a[j][j] = sqrt(dj);
        }
        __syncthreads();
        if (tid > j && tid < CB) a[tid][j] /= a[j][j];
        __syncthreads();
        for (int e = tid; e < CB * CB; e += 256) {
            const int i = e / CB, l = e % CB;
            if (l > j && l <= i) a[i][l] -= a[i][j] * a[l][j];
        }
        __syncthreads();
    }
    // column c of L^{-1} by forward substitution (thread c)
    if (tid < CB) {
        const int c = tid;
        for (int i = 0; i < c; ++i) x[i][c] = 0.0;
        for (int i = c; i < CB; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= a[i][k] * x[k][c];
            x[i][c] = s / a[i][i];
        }
    }
    __syncthreads();
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e / CB, l = e % CB;
        blk[(size_t)i * ld + l] = (l <= i) ? a[i][l] : 0.0;
        dinv[e] = x[i][l];
    }
}

// C (op)= A B^T over an inner dimension of 64: C is m x p (ld ldc), A m x 64
// (ld lda), B p x 64 (ld ldb), all row-major. One block per 64 x 64 tile of
// C (both operand tiles staged in LDS, so C may alias A: a block reads all of
// its rows before writing them); wave w computes rows 16 w.. of the tile
// against its four 16-column tiles. sub: C -= A B^T, else C = A B^T. lower:
// only tiles (ti, tj) with tj <= ti, numbered row by row.
__global__ __launch_bounds__(256) void gemm_nt_kernel(double* C, int ldc, const double* A, int lda,
                                                      const double* __restrict__ B, int ldb, int m, int p,
                                                      int sub, int lower) {
    __shared__ double as[CB][CLD];
    __shared__ double bs[CB][CLD];
    int ti, tj;
    if (lower) {
        // tile t = ti (ti + 1) / 2 + tj
        const int t = blockIdx.x;
        ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = blockIdx.x;
        tj = blockIdx.y;
    }
    const int i0 = ti * CB, j0 = tj * CB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < CB * CB; e += 256) {
        const int r = e / CB, k = e % CB;
        as[r][k] = (i0 + r < m) ? A[(size_t)(i0 + r) * lda + k] : 0.0;
        bs[r][k] = (j0 + r < p) ? B[(size_t)(j0 + r) * ldb + k] : 0.0;
    }
    __syncthreads();
    doublex4 acc[4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) acc[sb] = doublex4{0.0, 0.0, 0.0, 0.0};
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int st = 0; st < CB / 4; ++st) {
        const double av = as[wave * 16 + lr][4 * st + lk];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb)
            acc[sb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bs[sb * 16 + lr][4 * st + lk], acc[sb], 0, 0, 0);
    }
    // FP64 16x16x4 output: lane holds rows lane / 16 + 4 r of column lane % 16
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
        const int j = j0 + sb * 16 + lr;
        if (j >= p) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + wave * 16 + lk + 4 * r;
            if (i >= m) continue;
            double* c = C + (size_t)i * ldc + j;
            *c = sub ? *c - acc[sb][r] : acc[sb][r];
        }
    }
}

hipError_t gemm_nt(double* C, int ldc, const double* A, int lda, const double* B, int ldb, int m, int p, int sub,
                   int lower, hipStream_t st) {
    if (m <= 0 || p <= 0) return hipSuccess;
    const int tm = (m + CB - 1) / CB, tp = (p + CB - 1) / CB;
    if (lower) {
        const long long tiles = (long long)tm * (tm + 1) / 2;
        hipLaunchKernelGGL(gemm_nt_kernel, dim3((unsigned)tiles), dim3(256), 0, st, C, ldc, A, lda, B, ldb, m, p,
                           sub, 1);
    } else {
        hipLaunchKernelGGL(gemm_nt_kernel, dim3(tm, tp), dim3(256), 0, st, C, ldc, A, lda, B, ldb, m, p, sub, 0);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_chol_prep(double* A, int n, int npad, double shift, hipStream_t st) {
    hipLaunchKernelGGL(chol_prep_kernel, dim3((npad + 255) / 256), dim3(256), 0, st, A, n, npad, shift);
    return hipGetLastError();
}

hipError_t launch_chol_blocked(double* A, int npad, double* dinv, int* status, hipStream_t st) {
    if (npad <= 0 || npad % CB != 0) return hipErrorInvalidValue;
    const int nb = npad / CB;
    for (int k = 0; k < nb; ++k) {
        const int k0 = k * CB, rest = npad - k0 - CB;
        double* dk = dinv + (size_t)k * CB * CB;
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, st, A, npad, k0, dk, status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (rest == 0) break;
        double* below = A + (size_t)(k0 + CB) * npad + k0;          // L[k0 + 64.., k0..k0 + 63]
        e = gemm_nt(below, npad, below, npad, dk, CB, rest, CB, 0, 0, st);
        if (e != hipSuccess) return e;
        double* trail = A + (size_t)(k0 + CB) * npad + (k0 + CB);
        e = gemm_nt(trail, npad, below, npad, below, npad, rest, rest, 1, 1, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_trsm_right_lt(double* W, int rows, int npad, const double* L, const double* dinv, hipStream_t st) {
    if (npad <= 0 || npad % CB != 0) return hipErrorInvalidValue;
    const int nb = npad / CB;
    for (int k = 0; k < nb; ++k) {
        const int k0 = k * CB, rest = npad - k0 - CB;
        double* wk = W + k0;
        hipError_t e = gemm_nt(wk, npad, wk, npad, dinv + (size_t)k * CB * CB, CB, rows, CB, 0, 0, st);
        if (e != hipSuccess) return e;
        if (rest == 0) break;
        e = gemm_nt(W + k0 + CB, npad, wk, npad, L + (size_t)(k0 + CB) * npad + k0, npad, rows, rest, 1, 0, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ciq
