// Kernel products on MFMA (templates; instantiated per kernel type and
// lengthscale form in mvm_{f32,f64}_*.hip so the variants compile in parallel).
//  - FP32 path: FP32 kernel entries, v_mfma_f32_16x16x4_f32, FP64 running sums.
//  - FP64 path: FP64 kernel entries, v_mfma_f64_16x16x4_f64.
#pragma once

#include "ciq_internal.h"

#include <algorithm>

namespace ciq {
namespace mfma {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr float kLog2e = 1.4426950408889634f;

// FP32 kernel entry from r2 = sum_d (sc_d (x_d - x'_d))^2 with
//  RBF:      sc_d = 1/l_d        ->  k = exp(-r2/2) = 2^{-r2 log2(e)/2}
//  Matern52: sc_d = sqrt(5)/l_d  ->  rho = sqrt(r2), k = (1 + rho + rho^2/3) 2^{-rho log2 e}
template <int KERNEL>
__device__ __forceinline__ float kfun32(float r2) {
    if constexpr (KERNEL == CIQ_KERNEL_RBF) {
        return __builtin_amdgcn_exp2f(-0.5f * kLog2e * r2);
    } else {
        const float rho = __builtin_amdgcn_sqrtf(r2);
        const float e = __builtin_amdgcn_exp2f(-kLog2e * rho);
        return fmaf(rho, fmaf(rho, 1.0f / 3.0f, 1.0f), 1.0f) * e;
    }
}

__device__ __forceinline__ int done_now(const int* done) { return done != nullptr && *done != 0; }

// e^{-y} for y >= 0 in FP64 (within 1 ulp). e^{-y} = 2^n e^g with
// n = round(-y / ln2) and g = -y - n ln2, ln2 split in two parts (Cody-Waite)
// so that g carries no reduction error; |g| <= ln2/2. e^g is a degree-11
// polynomial fitted by the Remez exchange algorithm to minimise the maximum
// relative error on [-ln2/2, ln2/2] (3e-18 before rounding the coefficients;
// 1.6e-16 overall, checked in extended precision).
__device__ __forceinline__ double exp_neg(double y) {
    const double nf = rint(-y * 1.4426950408889634074);
    double g = fma(-nf, 6.93147180559945286227e-01, -y);
    g = fma(-nf, 2.31904681384629955842e-17, g);
    double p = 2.4994304884817207e-08;
    p = fma(p, g, 2.7632293279459877e-07);
    p = fma(p, g, 2.7557622530872255e-06);
    p = fma(p, g, 2.4801486521427463e-05);
    p = fma(p, g, 1.9841269432679237e-04);
    p = fma(p, g, 1.3888888951223987e-03);
    p = fma(p, g, 8.33333333355927e-03);
    p = fma(p, g, 4.166666666649277e-02);
    p = fma(p, g, 1.6666666666666170e-01);
    p = fma(p, g, 5.0000000000000180e-01);
    p = fma(p, g, 1.0);
    p = fma(p, g, 1.0);
    return ldexp(p, (int)fmax(nf, -1100.0));
}

// sqrt(x) for x >= 0 in FP64: hardware reciprocal square root, one
// Goldschmidt step for (sqrt x, 1/(2 sqrt x)) and two Newton corrections of
// the root. Inputs are clamped to 1e-200 so no scaling for subnormals or a
// zero special case is needed: the result for x = 0 is 1e-100, which leaves
// the Matern entry at exactly 1 in FP64.
__device__ __forceinline__ double sqrt64(double x) {
    x = fmax(x, 1e-200);
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}

// FP64 kernel entry from the scaled squared distance r2:
//   RBF:      r2 = sum_d ((x_d - x'_d)/l_d)^2,        k = e^{-r2/2}
//   Matern52: r2 = sum_d (sqrt5 (x_d - x'_d)/l_d)^2,  rho = sqrt(r2),
//             k = (1 + rho + rho^2/3) e^{-rho}
template <int KERNEL>
__device__ __forceinline__ double kentry64(double r2) {
    if constexpr (KERNEL == CIQ_KERNEL_RBF) {
        return exp_neg(0.5 * r2);
    } else {
        const double rho = sqrt64(r2);
        return (fma(r2, 1.0 / 3.0, 1.0) + rho) * exp_neg(rho);
    }
}

// ----------------------------------------------------------------------------
// FP32 kernel product on MFMA.
//
// Work decomposition: a block of 4 waves owns BM = 64*RT consecutive rows of
// one problem and one of `nsplit` contiguous ranges of columns j of K. Wave w
// owns rows [16*RT*w, 16*RT*(w+1)) of the block. Per 16 x 16 tile of K and
// per 16 columns of V, four v_mfma_f32_16x16x4_f32 cover the 16 j's: in step
// `st` lane l supplies A = K[i0 + l%16][j0 + 4*st + l/16] (computed in
// registers from its own x_i and the staged x_j) and
// B = V[j0 + 4*st + l/16][c0 + l%16] (from LDS); the accumulator holds
// Y[i0 + 4*(l/16) + r][c0 + l%16], r = 0..3.
//
// Batched runs (a.wl set): with a.queue the kernel is persistent -- a grid of
// the resident blocks, each taking work items (problem, row block, column
// range) from a global counter in list order (the host orders the list by
// problem size, largest first) until the list is exhausted; items of
// problems that have stopped are skipped. Without a.queue, block
// (x, y) does item (a.wl[x], split y).
//
// Accumulation: the MFMA accumulates one staged chunk of BN columns of K in
// FP32; each lane then adds its chunk sums into FP64 registers and restarts
// the FP32 accumulator. A plain FP32 accumulation over all N/nsplit columns
// loses ~sqrt(N) eps32 per output, and CIQ amplifies product errors by up to
// kappa(K); with the FP64 running sums the products carry only the rounding
// of the FP32 kernel entries and of short FP32 chunk sums.
// ----------------------------------------------------------------------------
template <int KERNEL, int DP, int NSB, int RT, bool ARD>
__device__ __forceinline__ void mvm_f32_item(const MvmArgs& a, const WorkItem* wip, int split, float* xs, float* vs) {
    constexpr int BM = 64 * RT;
    constexpr int BN = 64;
    constexpr int S16 = NSB * 16;
    constexpr int VST = (NSB & 1) ? S16 : S16 + 16;  // LDS row stride: rows j, j+1 hit disjoint banks
    constexpr int XE = BN * DP;                       // staged point doubles per chunk
    constexpr int XPT = (XE + 255) / 256;             // per thread
    constexpr int VPT = BN * S16 / 256;               // staged V floats per thread
    constexpr int VROWS = 256 / S16;                  // V rows covered by one pass of the block

    int n, off, rb;
    double o2, s2;
    float sc[DP];     // per-dimension scale applied to coordinate differences
    if (wip != nullptr) {
        const WorkItem wi = *wip;
        n = a.pn[wi.prob];
        off = a.poff[wi.prob];
        rb = wi.rb;
        o2 = a.po2[wi.prob];
        s2 = a.ps2[wi.prob];
#pragma unroll
        for (int k = 0; k < DP; ++k) sc[k] = (float)a.pscale[wi.prob * CIQ_MAX_D + k];
    } else {
        n = a.n;
        off = 0;
        rb = blockIdx.x;
        o2 = a.o2;
        s2 = a.s2;
#pragma unroll
        for (int k = 0; k < DP; ++k) sc[k] = (float)a.scale[k];
    }
    // isotropic: r^2 = sc0^2 * sum_d (x_d - x'_d)^2 (one multiply per entry)
    const float sc0sq = sc[0] * sc[0];
    const double* __restrict__ xh = static_cast<const double*>(a.xh) + (long long)off * DP;
    const float* __restrict__ v = static_cast<const float*>(a.v) + (long long)off * a.ldv;
    double* __restrict__ y = static_cast<double*>(a.y) + (long long)split * a.ysplit + (long long)off * a.ldy;
    const int s = a.s, ldv = a.ldv, ldy = a.ldy;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int row0 = rb * BM + wave * 16 * RT;

    float xi[RT][DP];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int i = row0 + rt * 16 + (lane & 15);
#pragma unroll
        for (int k = 0; k < DP; ++k) xi[rt][k] = (i < n) ? (float)xh[(long long)i * DP + k] : 0.0f;
    }

    // narrow launches (<= 32 columns) rotate four FP32 accumulators over the
    // chunk's 4-column steps: each FP32 sum spans 16 columns, not 64
    constexpr int NACC = (NSB <= 2) ? 4 : 1;
    floatx4 acc[NACC][RT][NSB];
    double accd[RT][NSB][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
#pragma unroll
            for (int h = 0; h < NACC; ++h) acc[h][rt][sb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) accd[rt][sb][r] = 0.0;
        }

    const int nchunk = (n + BN - 1) / BN;
    const int c0 = (int)(((long long)split * nchunk) / a.nsplit);
    const int c1 = (int)(((long long)(split + 1) * nchunk) / a.nsplit);

    // register staging of the next chunk (loads in flight while the current
    // chunk is computed); each thread owns fixed (row, column) slots
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
#pragma unroll
        for (int k = 0; k < VPT; ++k) vs[(vr + k * VROWS) * VST + vc] = vreg[k];
        __syncthreads();
        if (c + 1 < c1) fetch(c + 1);
#pragma unroll
        for (int jb = 0; jb < BN / 16; ++jb) {
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int jl = jb * 16 + st * 4 + (lane >> 4);
                float xj[DP];
#pragma unroll
                for (int k = 0; k < DP; ++k) xj[k] = xs[jl * DP + k];
                float kv[RT];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    // raw-coordinate differences first (exact for close
                    // points), the lengthscale scaling after
                    float r2 = 0.0f;
#pragma unroll
                    for (int k = 0; k < DP; ++k) {
                        const float dd = xi[rt][k] - xj[k];
                        if constexpr (ARD) {
                            const float u = dd * sc[k];
                            r2 = fmaf(u, u, r2);
                        } else {
                            r2 = fmaf(dd, dd, r2);
                        }
                    }
                    if constexpr (!ARD) r2 *= sc0sq;
                    kv[rt] = kfun32<KERNEL>(r2);
                }
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb) {
                    const float bv = vs[jl * VST + sb * 16 + (lane & 15)];
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[st % NACC][rt][sb] =
                            __builtin_amdgcn_mfma_f32_16x16x4f32(kv[rt], bv, acc[st % NACC][rt][sb], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < NACC; ++h)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) accd[rt][sb][r] += (double)acc[h][rt][sb][r];
                    acc[h][rt][sb] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
    }

#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
            const int cc = sb * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = row0 + rt * 16 + 4 * (lane >> 4) + r;
                if (i < n && cc < s) {
                    double val = o2 * accd[rt][sb][r];
                    if (split == 0) val = fma(s2, (double)v[(long long)i * ldv + cc], val);
                    y[(long long)i * ldy + cc] = val;
                }
            }
        }
    }
}

template <int KERNEL, int DP, int NSB, int RT, bool ARD>
__global__ __launch_bounds__(256) void mvm_f32_kernel(MvmArgs a) {
    constexpr int S16 = NSB * 16;
    constexpr int VST = (NSB & 1) ? S16 : S16 + 16;
    __shared__ float xs[64 * DP];
    __shared__ float vs[64 * VST];
    __shared__ int item_sh;
    if (done_now(a.done)) return;
    if (a.queue != nullptr) {           // persistent: items from the global counter
        for (;;) {
            __syncthreads();            // every thread has read the previous item
            if (threadIdx.x == 0) item_sh = atomicAdd(a.queue, 1);
            __syncthreads();
            const int item = item_sh;
            if (item >= a.nitems) break;
            const WorkItem* wip = a.wl + item / a.nsplit;
            if (a.prob_done != nullptr && a.prob_done[wip->prob]) continue;
            mvm_f32_item<KERNEL, DP, NSB, RT, ARD>(a, wip, item % a.nsplit, xs, vs);
        }
        return;
    }
    const WorkItem* wip = (a.wl != nullptr) ? a.wl + blockIdx.x : nullptr;
    if (wip != nullptr && a.prob_done != nullptr && a.prob_done[wip->prob]) return;
    mvm_f32_item<KERNEL, DP, NSB, RT, ARD>(a, wip, blockIdx.y, xs, vs);
}

// blocks of a kernel variant one CU holds (0 if the runtime cannot say)
template <typename K>
inline int resident_blocks_per_cu(K kernel) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

template <int KERNEL, int DP, int NSB, int RT, bool ARD>
hipError_t launch_f32_variant(const MvmArgs& a, int grid_x, hipStream_t st) {
    if (a.queue != nullptr) {
        // persistent grid: the blocks the device holds at once (cached per variant)
        static int slots = 0;
        if (slots == 0) {
            int dev = 0, ncu = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
                slots = std::max(1, resident_blocks_per_cu(mvm_f32_kernel<KERNEL, DP, NSB, RT, ARD>)) * ncu;
            else
                slots = 1024;
            (void)hipGetLastError();
        }
        const hipError_t e = launch_fill<int>(a.queue, 1, 0, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((mvm_f32_kernel<KERNEL, DP, NSB, RT, ARD>), dim3(std::min(a.nitems, slots)), dim3(256), 0,
                           st, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((mvm_f32_kernel<KERNEL, DP, NSB, RT, ARD>), dim3(grid_x, a.nsplit), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int KERNEL, bool ARD, int DP, int NSB>
hipError_t launch_f32_nsb(const MvmArgs& a, int grid_x, hipStream_t st) {
    if constexpr (NSB >= 8) {
        return launch_f32_variant<KERNEL, DP, NSB, 1, ARD>(a, grid_x, st);
    } else {
        if (a.rt == 1) return launch_f32_variant<KERNEL, DP, NSB, 1, ARD>(a, grid_x, st);
        return launch_f32_variant<KERNEL, DP, NSB, 2, ARD>(a, grid_x, st);
    }
}

template <int KERNEL, bool ARD, int DP>
hipError_t launch_f32_dp(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    switch (nsb) {
        case 1: return launch_f32_nsb<KERNEL, ARD, DP, 1>(a, grid_x, st);
        case 2: return launch_f32_nsb<KERNEL, ARD, DP, 2>(a, grid_x, st);
        case 3:
        case 4: return launch_f32_nsb<KERNEL, ARD, DP, 4>(a, grid_x, st);
        default: return launch_f32_nsb<KERNEL, ARD, DP, 8>(a, grid_x, st);
    }
}

template <int KERNEL, bool ARD>
hipError_t launch_f32_k(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    switch (a.dp) {
        case 4: return launch_f32_dp<KERNEL, ARD, 4>(a, nsb, grid_x, st);
        case 6: return launch_f32_dp<KERNEL, ARD, 6>(a, nsb, grid_x, st);
        case 8: return launch_f32_dp<KERNEL, ARD, 8>(a, nsb, grid_x, st);
        case 10: return launch_f32_dp<KERNEL, ARD, 10>(a, nsb, grid_x, st);
        case 12: return launch_f32_dp<KERNEL, ARD, 12>(a, nsb, grid_x, st);
        default: return launch_f32_dp<KERNEL, ARD, 16>(a, nsb, grid_x, st);
    }
}


// ----------------------------------------------------------------------------
// FP64 kernel product on MFMA (v_mfma_f64_16x16x4_f64).
//
// Same decomposition as the FP32 kernel: a block of 4 waves owns 64*RT rows
// and one range of columns j; per staged chunk of 64 j's, each lane evaluates
// the FP64 entries of its A-operand K[i0 + l%16][j0 + 4*step + l/16], the
// B-operand is V[j0 + 4*step + l/16][c0 + l%16]. The FP64 16x16x4 MFMA leaves
// Y[i0 + l/16 + 4r][c0 + l%16] in register r (lane layout verified on gfx950).
// Everything is FP64: entries, products, accumulation.
// ----------------------------------------------------------------------------
template <int KERNEL, int DP, int NSB, int RT, bool ARD>
__global__ __launch_bounds__(256) void mvm_f64mfma_kernel(MvmArgs a) {
    constexpr int BM = 64 * RT;
    constexpr int BN = 64;
    constexpr int S16 = NSB * 16;
    constexpr int VST = (NSB & 1) ? S16 : S16 + 16;   // rows j, j+1 on disjoint banks
    constexpr int XE = BN * DP;
    constexpr int XPT = (XE + 255) / 256;
    constexpr int VPT = BN * S16 / 256;
    constexpr int VROWS = 256 / S16;
    __shared__ double xs[XE];
    __shared__ double vs[BN * VST];

    if (done_now(a.done)) return;
    int n, off, rb;
    double o2, s2;
    double sc[DP];
    if (a.wl != nullptr) {
        const WorkItem wi = a.wl[blockIdx.x];
        if (a.prob_done != nullptr && a.prob_done[wi.prob]) return;
        n = a.pn[wi.prob];
        off = a.poff[wi.prob];
        rb = wi.rb;
        o2 = a.po2[wi.prob];
        s2 = a.ps2[wi.prob];
#pragma unroll
        for (int k = 0; k < DP; ++k) sc[k] = a.pscale[wi.prob * CIQ_MAX_D + k];
    } else {
        n = a.n;
        off = 0;
        rb = blockIdx.x;
        o2 = a.o2;
        s2 = a.s2;
#pragma unroll
        for (int k = 0; k < DP; ++k) sc[k] = a.scale[k];
    }
    const double sc0sq = sc[0] * sc[0];
    const int split = blockIdx.y;
    const double* __restrict__ xh = static_cast<const double*>(a.xh) + (long long)off * DP;
    const double* __restrict__ v = static_cast<const double*>(a.v) + (long long)off * a.ldv;
    double* __restrict__ y = static_cast<double*>(a.y) + (long long)split * a.ysplit + (long long)off * a.ldy;
    const int s = a.s, ldv = a.ldv, ldy = a.ldy;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int row0 = rb * BM + wave * 16 * RT;

    double xi[RT][DP];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int i = row0 + rt * 16 + (lane & 15);
#pragma unroll
        for (int k = 0; k < DP; ++k) xi[rt][k] = (i < n) ? xh[(long long)i * DP + k] : 0.0;
    }

    doublex4 acc[RT][NSB];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) acc[rt][sb] = doublex4{0.0, 0.0, 0.0, 0.0};

    const int nchunk = (n + BN - 1) / BN;
    const int c0 = (int)(((long long)split * nchunk) / a.nsplit);
    const int c1 = (int)(((long long)(split + 1) * nchunk) / a.nsplit);

    const int vr = tid / S16, vc = tid - (tid / S16) * S16;
    const bool vcol_ok = vc < s;
    double xreg[XPT], vreg[VPT];
    auto fetch = [&](int c) {
        const int j0 = c * BN;
#pragma unroll
        for (int k = 0; k < XPT; ++k) {
            const int e = tid + 256 * k;
            const int j = j0 + e / DP;
            xreg[k] = (e < XE && j < n) ? xh[(long long)j0 * DP + e] : 0.0;
        }
        const double* vp = v + (long long)(j0 + vr) * ldv + vc;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int j = j0 + vr + k * VROWS;
            vreg[k] = (vcol_ok && j < n) ? vp[(long long)k * VROWS * ldv] : 0.0;
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
#pragma unroll
        for (int k = 0; k < VPT; ++k) vs[(vr + k * VROWS) * VST + vc] = vreg[k];
        __syncthreads();
        if (c + 1 < c1) fetch(c + 1);
#pragma unroll
        for (int jb = 0; jb < BN / 16; ++jb) {
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int jl = jb * 16 + st * 4 + (lane >> 4);
                double xj[DP];
#pragma unroll
                for (int k = 0; k < DP; ++k) xj[k] = xs[jl * DP + k];
                double kv[RT];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    double r2 = 0.0;
#pragma unroll
                    for (int k = 0; k < DP; ++k) {
                        const double dd = xi[rt][k] - xj[k];
                        if constexpr (ARD) {
                            const double u = dd * sc[k];
                            r2 = fma(u, u, r2);
                        } else {
                            r2 = fma(dd, dd, r2);
                        }
                    }
                    if constexpr (!ARD) r2 *= sc0sq;
                    kv[rt] = kentry64<KERNEL>(r2);
                }
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb) {
                    const double bv = vs[jl * VST + sb * 16 + (lane & 15)];
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[rt][sb] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv[rt], bv, acc[rt][sb], 0, 0, 0);
                }
            }
        }
    }

#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
            const int cc = sb * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = row0 + rt * 16 + (lane >> 4) + 4 * r;
                if (i < n && cc < s) {
                    double val = o2 * acc[rt][sb][r];
                    if (split == 0) val = fma(s2, v[(long long)i * ldv + cc], val);
                    y[(long long)i * ldy + cc] = val;
                }
            }
        }
    }
}

template <int KERNEL, bool ARD, int DP, int NSB>
hipError_t launch_f64m_nsb(const MvmArgs& a, int grid_x, hipStream_t st) {
    dim3 grid(grid_x, a.nsplit);
    if (a.rt == 1)
        hipLaunchKernelGGL((mvm_f64mfma_kernel<KERNEL, DP, NSB, 1, ARD>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((mvm_f64mfma_kernel<KERNEL, DP, NSB, 2, ARD>), grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int KERNEL, bool ARD, int DP>
hipError_t launch_f64m_dp(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    switch (nsb) {
        case 1: return launch_f64m_nsb<KERNEL, ARD, DP, 1>(a, grid_x, st);
        case 2: return launch_f64m_nsb<KERNEL, ARD, DP, 2>(a, grid_x, st);
        default: return launch_f64m_nsb<KERNEL, ARD, DP, 4>(a, grid_x, st);
    }
}

template <int KERNEL, bool ARD>
hipError_t launch_f64m_k(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    switch (a.dp) {
        case 4: return launch_f64m_dp<KERNEL, ARD, 4>(a, nsb, grid_x, st);
        case 6: return launch_f64m_dp<KERNEL, ARD, 6>(a, nsb, grid_x, st);
        case 8: return launch_f64m_dp<KERNEL, ARD, 8>(a, nsb, grid_x, st);
        case 10: return launch_f64m_dp<KERNEL, ARD, 10>(a, nsb, grid_x, st);
        case 12: return launch_f64m_dp<KERNEL, ARD, 12>(a, nsb, grid_x, st);
        default: return launch_f64m_dp<KERNEL, ARD, 16>(a, nsb, grid_x, st);
    }
}

}  // namespace mfma
}  // namespace ciq
