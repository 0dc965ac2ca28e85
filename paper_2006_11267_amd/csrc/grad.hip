// Hyperparameter part of the CIQ backward pass (Sec. 3.3).
//
// With a_q = (t_q I + K)^{-1} B (forward solves) and g_q = (t_q I + K)^{-1} G'
// (backward solves), the gradient of <G, out> with respect to K is
// -1/2 sum_q w_q (g_q a_q^T + a_q g_q^T) (+ 1/2 (G A^T + A G^T) for the square
// root). Contracted with a symmetric dK/dtheta this is
//     dL/dtheta = - sum_ij W_ij dK_ij/dtheta,   W_ij = U_i . V_j,
// U_i = [w_1 g_1(i,:), ..., w_Q g_Q(i,:), (-G(i,:))],
// V_j = [a_1(j,:), ..., a_Q(j,:), (A(j,:))].
// The tile pass forms W block by block on FP64 MFMA (v_mfma_f64_16x16x4_f64)
// and reduces it against dK/dtheta evaluated in registers; no N x N matrix
// is stored. dK/dtheta (u = x / l per dimension, r^2 = |u_i - u_j|^2):
//   d/d outputscale:  k(r)
//   d/d noise:        delta_ij
//   d/d l_d:          o^2 h(r) (u_id - u_jd)^2 / l_d,
//                     h = k (RBF), h = (5/3)(1 + sqrt5 r) exp(-sqrt5 r) (Matern-5/2).
#include "ciq_internal.h"

#include <cmath>

namespace ciq {

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;      // contraction chunk staged per LDS round
constexpr int TM = 64;      // rows (i) per block
constexpr int TN = 64;      // columns (j) per block
constexpr double kSqrt5d = 2.23606797749978969640917366873;

// U[i][k], V[i][k] with k = q*s + c (+ Q*s + c for the square-root block),
// rows padded to rows_pad and k padded to kpad with zeros.
template <typename T>
__global__ void build_uv_kernel(const double* gq, const T* aq, const T* g, int ldg, const double* w, int n,
                                int Q, int s, int sqrt_mode, int kpad, int rows_pad, double* U, double* V) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows_pad * kpad) return;
    const int i = (int)(e / kpad), k = (int)(e - (long long)i * kpad);
    double u = 0.0, v = 0.0;
    if (i < n) {
        if (k < Q * s) {
            const int q = k / s, c = k - q * s;
            u = w[q] * gq[((long long)i * Q + q) * s + c];
            v = (double)aq[((long long)i * Q + q) * s + c];
        } else if (sqrt_mode && k < (Q + 1) * s) {
            const int c = k - Q * s;
            u = -(double)g[(long long)i * ldg + c];
            double a = 0.0;
            for (int q = 0; q < Q; ++q) a += w[q] * (double)aq[((long long)i * Q + q) * s + c];
            v = a;
        }
    }
    U[e] = u;
    V[e] = v;
}

template <int KERNEL, int DP>
__global__ __launch_bounds__(256) void grad_tiles_kernel(const double* U, const double* V, int kpad,
                                                          const double* pts, int n, int nd,
                                                          double* partial) {
    // LDS: U block [TM][KC+1], V block [TN][KC+1], points of the i and j blocks
    __shared__ double su[TM * (KC + 1)];
    __shared__ double sv[TN * (KC + 1)];
    __shared__ double pi_[TM * DP];
    __shared__ double pj_[TN * DP];
    __shared__ double red[4][DP + 2];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;   // wave's 32 x 32 sub-block

    for (int e = threadIdx.x; e < TM * DP; e += 256) {
        const int r = e / DP, k = e - r * DP;
        pi_[e] = (i0 + r < n) ? pts[(long long)(i0 + r) * DP + k] : 0.0;
        pj_[e] = (j0 + r < n) ? pts[(long long)(j0 + r) * DP + k] : 0.0;
    }

    doublex4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = doublex4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < kpad; k0 += KC) {
        __syncthreads();
        for (int e = threadIdx.x; e < TM * KC; e += 256) {
            const int r = e / KC, k = e - r * KC;
            su[r * (KC + 1) + k] = U[(long long)(i0 + r) * kpad + k0 + k];
            sv[r * (KC + 1) + k] = V[(long long)(j0 + r) * kpad + k0 + k];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            const int kl = kk + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = su[(wi + 16 * a + (lane & 15)) * (KC + 1) + kl];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = sv[(wj + 16 * b + (lane & 15)) * (KC + 1) + kl];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }

    // epilogue: the FP64 16x16x4 MFMA leaves W[i][j] in lane l, register r for
    // i = wi + 16a + l/16 + 4r, j = wj + 16b + l%16 (checked on gfx950 with an
    // in-bounds layout probe; the FP32 16x16x4 layout differs: i = 4(l/16) + r)
    double g[DP + 2];
#pragma unroll
    for (int k = 0; k < DP + 2; ++k) g[k] = 0.0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int jl = wj + 16 * b + (lane & 15);
        double uj[DP];
#pragma unroll
        for (int k = 0; k < DP; ++k) uj[k] = pj_[jl * DP + k];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int il = wi + 16 * a + (lane >> 4) + 4 * r;
                const int i = i0 + il, j = j0 + jl;
                if (i >= n || j >= n) continue;
                const double wij = acc[a][b][r];
                double diff2[DP];
                double r2 = 0.0;
#pragma unroll
                for (int k = 0; k < DP; ++k) {
                    const double dd = pi_[il * DP + k] - uj[k];
                    diff2[k] = dd * dd;
                    r2 += diff2[k];
                }
                double kv, h;
                if constexpr (KERNEL == CIQ_KERNEL_RBF) {
                    kv = exp(-0.5 * r2);
                    h = kv;
                } else {
                    const double rho = kSqrt5d * sqrt(r2);
                    const double ex = exp(-rho);
                    kv = (1.0 + rho + rho * rho * (1.0 / 3.0)) * ex;
                    h = (5.0 / 3.0) * (1.0 + rho) * ex;
                }
                const double wh = wij * h;
#pragma unroll
                for (int k = 0; k < DP; ++k) g[k] = fma(wh, diff2[k], g[k]);
                g[DP] = fma(wij, kv, g[DP]);
                if (i == j) g[DP + 1] += wij;
            }
        }
    }
    // wave reduction (fixed butterfly order), then the 4 waves in order
#pragma unroll
    for (int k = 0; k < DP + 2; ++k) {
        double v = g[k];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        g[k] = v;
    }
    if (lane == 0)
        for (int k = 0; k < DP + 2; ++k) red[wave][k] = g[k];
    __syncthreads();
    if (threadIdx.x < DP + 2) {
        const int k = threadIdx.x;
        const double sum = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        partial[((long long)blockIdx.y * gridDim.x + blockIdx.x) * (DP + 2) + k] = sum;
    }
    (void)nd;
}

template <int KERNEL>
hipError_t launch_grad_k(const double* U, const double* V, int kpad, const double* pts, int n, int dp, int nd,
                         double* partial, dim3 grid, hipStream_t st) {
    switch (dp) {
        case 4:
            hipLaunchKernelGGL((grad_tiles_kernel<KERNEL, 4>), grid, dim3(256), 0, st, U, V, kpad, pts, n, nd, partial);
            break;
        case 8:
            hipLaunchKernelGGL((grad_tiles_kernel<KERNEL, 8>), grid, dim3(256), 0, st, U, V, kpad, pts, n, nd, partial);
            break;
        case 12:
            hipLaunchKernelGGL((grad_tiles_kernel<KERNEL, 12>), grid, dim3(256), 0, st, U, V, kpad, pts, n, nd, partial);
            break;
        default:
            hipLaunchKernelGGL((grad_tiles_kernel<KERNEL, 16>), grid, dim3(256), 0, st, U, V, kpad, pts, n, nd, partial);
            break;
    }
    return hipGetLastError();
}

}  // namespace

int grad_rows_pad(int n) { return ((n + 63) / 64) * 64; }
int grad_k_pad(int k) { return ((k + KC - 1) / KC) * KC; }

template <typename T>
hipError_t launch_build_uv(const double* gq, const T* aq, const T* g, int ldg, const double* w_dev, int n, int Q,
                           int s, int sqrt_mode, double* U, double* V, hipStream_t st) {
    const int kpad = grad_k_pad((Q + (sqrt_mode ? 1 : 0)) * s);
    const int rows = grad_rows_pad(n);
    const long long total = (long long)rows * kpad;
    hipLaunchKernelGGL(build_uv_kernel<T>, dim3((int)((total + 255) / 256)), dim3(256), 0, st, gq, aq, g, ldg,
                       w_dev, n, Q, s, sqrt_mode, kpad, rows, U, V);
    return hipGetLastError();
}
template hipError_t launch_build_uv<float>(const double*, const float*, const float*, int, const double*, int, int,
                                           int, int, double*, double*, hipStream_t);
template hipError_t launch_build_uv<double>(const double*, const double*, const double*, int, const double*, int,
                                            int, int, int, double*, double*, hipStream_t);

hipError_t launch_grad_pass(int kernel, const double* U, const double* V, int kpad, const double* pts, int n,
                            int dp, double* partial, int* nblocks, hipStream_t st) {
    const int nb = grad_rows_pad(n) / 64;
    dim3 grid(nb, nb);
    *nblocks = nb * nb;
    return kernel == CIQ_KERNEL_RBF ? launch_grad_k<CIQ_KERNEL_RBF>(U, V, kpad, pts, n, dp, dp, partial, grid, st)
                                    : launch_grad_k<CIQ_KERNEL_MATERN52>(U, V, kpad, pts, n, dp, dp, partial, grid, st);
}

}  // namespace ciq
