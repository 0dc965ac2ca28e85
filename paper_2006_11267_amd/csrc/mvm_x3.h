// Split-operand half-precision kernel product (precision forms CIQ_BF16X3 and
// CIQ_F16X3; templates instantiated in mvm_x3_{rbf,m52}.hip).
//
// Entries are evaluated in FP32 from raw-coordinate differences (as in the
// FP32 product) and every operand is split into two 16-bit parts,
//     e = e_hi + 2^-SC e_lo',   e_hi = h(e),  e_lo' = h((e - e_hi) 2^SC),
// h() the rounding to BF16 (SC = 8) or FP16 (SC = 11); the lower part is
// scaled up so it stays in FP16's normal range. One product is then
//     K V ~ K_hi V_hi + 2^-SC (K_hi V_lo' + K_lo' V_hi)
// on v_mfma_f32_16x16x32_{bf16,f16} with two FP32 accumulators (the
// K_lo V_lo term, ~2^-2SC relative, is dropped), flushed into FP64 after every
// 64-column chunk. Relative error per product ~2^-(SC+8) for BF16 (~1e-5) and
// the FP32 entry rounding for FP16 (~1e-6).
//
// MFMA lane layout (16x16x32, 8 values per lane): lane l holds A[i = l%16][k]
// and B[k][j = l%16] for eight k of the group l/16 (any fixed assignment of k
// to (l/16, v) works, as long as A and B use the same); the accumulator holds
// Y[4(l/16) + r][l%16], r = 0..3 (checked on gfx950 with an in-bounds probe).
// Here k = 8(l/16) + v.
#pragma once

#include "mvm_mfma.h"

namespace ciq {
namespace x3 {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <bool HALF>
struct Half;
template <>
struct Half<false> {
    typedef __bf16 T;
    typedef bf16x8 V8;
    static constexpr float kUp = 256.0f;          // 2^8
    static constexpr float kDown = 1.0f / 256.0f;
    static __device__ __forceinline__ floatx4 mfma(V8 a, V8 b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Half<true> {
    typedef _Float16 T;
    typedef f16x8 V8;
    static constexpr float kUp = 2048.0f;         // 2^11
    static constexpr float kDown = 1.0f / 2048.0f;
    static __device__ __forceinline__ floatx4 mfma(V8 a, V8 b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <int KERNEL, int DP, int NSB, bool ARD, bool HALF>
__global__ __launch_bounds__(256) void mvm_x3_kernel(MvmArgs a) {
    using H = Half<HALF>;
    using T = typename H::T;
    constexpr int BN = 64;                // columns j per staged chunk (two MFMA steps of 32)
    constexpr int S16 = NSB * 16;
    constexpr int JST = BN + 8;           // LDS row stride of the transposed V parts (16-byte rows)
    constexpr int XE = BN * DP;
    constexpr int XPT = (XE + 255) / 256;
    constexpr int VPT = BN * S16 / 256;
    constexpr int VROWS = 256 / S16;
    __shared__ float xs[XE];
    __shared__ __attribute__((aligned(16))) T vh[S16 * JST];
    __shared__ __attribute__((aligned(16))) T vl[S16 * JST];

    if (mfma::done_now(a.done)) return;
    const int n = a.n;
    const double o2 = a.o2, s2 = a.s2;
    float sc[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) sc[k] = (float)a.scale[k];
    const float sc0sq = sc[0] * sc[0];
    const int rb = blockIdx.x, split = blockIdx.y;
    const double* __restrict__ xh = static_cast<const double*>(a.xh);
    const float* __restrict__ v = static_cast<const float*>(a.v);
    double* __restrict__ y = static_cast<double*>(a.y) + (long long)split * a.ysplit;
    const int s = a.s, ldv = a.ldv, ldy = a.ldy;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row0 = rb * 64 + wave * 16;
    float xi[DP];
    {
        const int i = row0 + (lane & 15);
#pragma unroll
        for (int k = 0; k < DP; ++k) xi[k] = (i < n) ? (float)xh[(long long)i * DP + k] : 0.0f;
    }

    floatx4 ahh[NSB], ax[NSB];
    double accd[NSB][4];
#pragma unroll
    for (int sb = 0; sb < NSB; ++sb) {
        ahh[sb] = floatx4{0.f, 0.f, 0.f, 0.f};
        ax[sb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) accd[sb][r] = 0.0;
    }

    const int nchunk = (n + BN - 1) / BN;
    const int c0 = (int)(((long long)split * nchunk) / a.nsplit);
    const int c1 = (int)(((long long)(split + 1) * nchunk) / a.nsplit);

    const int vr = tid / S16, vc = tid - (tid / S16) * S16;
    const bool vcol_ok = vc < s;
    float xreg[XPT], vreg[VPT];
    auto fetch = [&](int c) {
        const int j0 = c * BN;
#pragma unroll
        for (int k = 0; k < XPT; ++k) {
            const int e = tid + 256 * k;
            const int j = j0 + e / DP;
            xreg[k] = (e < XE && j < n) ? (float)xh[(long long)j0 * DP + e] : 0.0f;
        }
        const float* vp = v + (long long)(j0 + vr) * ldv + vc;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int j = j0 + vr + k * VROWS;
            vreg[k] = (vcol_ok && j < n) ? vp[(long long)k * VROWS * ldv] : 0.0f;
        }
    };
    if (c0 < c1) fetch(c0);

    for (int c = c0; c < c1; ++c) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < XPT; ++k) {
            const int e = tid + 256 * k;
            if (e < XE) xs[e] = xreg[k];
        }
        // V parts, transposed: [column][row of the chunk]
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const float x = vreg[k];
            const T hi = (T)x;
            const T lo = (T)((x - (float)hi) * H::kUp);
            vh[vc * JST + vr + k * VROWS] = hi;
            vl[vc * JST + vr + k * VROWS] = lo;
        }
        __syncthreads();
        if (c + 1 < c1) fetch(c + 1);
#pragma unroll
        for (int jb = 0; jb < BN / 32; ++jb) {
            const int jg = jb * 32 + 8 * (lane >> 4);    // this lane's 8 columns j of the step
            typename H::V8 kh, kl;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                float r2 = 0.0f;
#pragma unroll
                for (int k = 0; k < DP; ++k) {
                    const float dd = xi[k] - xs[(jg + u) * DP + k];
                    if constexpr (ARD) {
                        const float w = dd * sc[k];
                        r2 = fmaf(w, w, r2);
                    } else {
                        r2 = fmaf(dd, dd, r2);
                    }
                }
                if constexpr (!ARD) r2 *= sc0sq;
                const float e = mfma::kfun32<KERNEL>(r2);
                const T hi = (T)e;
                kh[u] = hi;
                kl[u] = (T)((e - (float)hi) * H::kUp);
            }
#pragma unroll
            for (int sb = 0; sb < NSB; ++sb) {
                const int off = (sb * 16 + (lane & 15)) * JST + jg;
                const typename H::V8 bh = *reinterpret_cast<const typename H::V8*>(&vh[off]);
                const typename H::V8 bl = *reinterpret_cast<const typename H::V8*>(&vl[off]);
                ahh[sb] = H::mfma(kh, bh, ahh[sb]);
                ax[sb] = H::mfma(kh, bl, ax[sb]);
                ax[sb] = H::mfma(kl, bh, ax[sb]);
            }
        }
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                accd[sb][r] += (double)ahh[sb][r] + (double)ax[sb][r] * (double)H::kDown;
            ahh[sb] = floatx4{0.f, 0.f, 0.f, 0.f};
            ax[sb] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    }

#pragma unroll
    for (int sb = 0; sb < NSB; ++sb) {
        const int cc = sb * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = row0 + 4 * (lane >> 4) + r;
            if (i < n && cc < s) {
                double val = o2 * accd[sb][r];
                if (split == 0) val = fma(s2, (double)v[(long long)i * ldv + cc], val);
                y[(long long)i * ldy + cc] = val;
            }
        }
    }
}

template <int KERNEL, bool ARD, bool HALF, int DP>
hipError_t launch_x3_dp(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    dim3 grid(grid_x, a.nsplit);
    switch (nsb) {
        case 1: hipLaunchKernelGGL((mvm_x3_kernel<KERNEL, DP, 1, ARD, HALF>), grid, dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((mvm_x3_kernel<KERNEL, DP, 2, ARD, HALF>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((mvm_x3_kernel<KERNEL, DP, 4, ARD, HALF>), grid, dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

template <int KERNEL, bool ARD, bool HALF>
hipError_t launch_x3_k(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    switch (a.dp) {
        case 4: return launch_x3_dp<KERNEL, ARD, HALF, 4>(a, nsb, grid_x, st);
        case 8: return launch_x3_dp<KERNEL, ARD, HALF, 8>(a, nsb, grid_x, st);
        case 12: return launch_x3_dp<KERNEL, ARD, HALF, 12>(a, nsb, grid_x, st);
        default: return launch_x3_dp<KERNEL, ARD, HALF, 16>(a, nsb, grid_x, st);
    }
}

}  // namespace x3
}  // namespace ciq
