// Resident kernel matrix for the FP64 path.
//
// msMINRES applies the same K in every iteration (Sec. 3.2). Evaluating the
// entries costs ~49 FP64 VALU instructions per 64 entries on gfx950, and the
// FP64 VALU shares its datapath with the FP64 MFMA (no overlap), so an
// on-the-fly product pays entry generation plus contraction in every
// iteration. When the matrix fits in device memory (N = 50,000 in FP64 is
// 20 GB of the 288 GB), one build pass writes the unit-scale entries k(x_i, x_j)
// once per call and every product streams them from HBM; the loads overlap
// with the MFMA contraction, which is then the only bound.
//
// Layout ("operand-tiled"): with ib = i / 16, js = j / 4 (the 4-column step)
// and lane = (i % 16) + 16 * (j % 4), the entry K[i][j] sits at
//     kt[((ib * (njs / 2) + js / 2) * 64 + lane) * 2 + js % 2],
// njs = padded columns / 4. One 64-lane load of 16 bytes per lane returns,
// in lane l, the A-operands of v_mfma_f64_16x16x4_f64 for two consecutive
// steps, K[16 ib + l % 16][4 js + l / 16] for js = 2p, 2p + 1, from 1 KB of
// contiguous memory (16-byte lanes stream measurably faster than 8-byte
// ones). Rows are padded to a multiple of 128 and columns to a multiple of 64;
// the padding holds finite entries of zero points, which meet zero rows of V.
//
// The FP32 path keeps the same entries rounded once to FP32 (10 GB at
// N = 50,000) in the same order with four steps per 16-byte lane:
//     kt32[((ib * (njs / 4) + js / 4) * 64 + lane) * 4 + js % 4],
// and contracts them on v_mfma_f32_16x16x4_f32, whose A-operand lane layout
// is the FP64 one. FP64 entries rounded once are ~10x more accurate than the
// FP32 evaluation the on-the-fly FP32 product uses.
//
// The split FP16 form (CIQ_F16X3) stores every FP64 entry k as two halves,
// hi = fp16(k) and lo = fp16((k - hi) 2^11) (4 bytes per entry, like FP32),
// in the A-operand order of v_mfma_f32_16x16x32_f16: for the 16-row tile ib
// and the k-step ks (32 columns), 64 lanes x 8 halfs of hi then of lo, lane l
// holding K[16 ib + l % 16][32 ks + 8 (l / 16) + v], v = 0..7:
//     kt16[(((ib * nks + ks) * 2 + part) * 64 + lane) * 8 + v],  nks = padded columns / 32.
// Unit-scale entries lie in [0, 1]: hi + 2^-11 lo carries 22 significant
// bits (absolute error <= 2^-22 |k| for normal hi, ~1e-11 below FP16's
// normal range). The product multiplies the split operand vh + 2^-11 vl
// (op16_index layout) by three part pairs,
//     K V ~ Kh Vh + 2^-11 (Kh Vl + Kl Vh),
// on v_mfma_f32_16x16x32_f16 with FP32 accumulators (the hi x hi sum flushed
// into FP64 after every 64-column chunk); the dropped 2^-22 Kl Vl term is
// ~2^-24 relative, below the 22-bit representation error. Its bytes per entry
// equal the FP32 form's while its MFMA work is a seventh, so it streams K at
// close to HBM speed.
#include "mvm_mfma.h"

namespace ciq {
namespace {

using mfma::doublex4;
using mfma::floatx4;
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ---- build pass ------------------------------------------------------------
// grid.x: 64-row blocks (one 16-row tile per wave), grid.y: column ranges.
template <int KERNEL, int DP, bool ARD, int ELEM>
__global__ __launch_bounds__(256) void kbuild_kernel(KBuildArgs a) {
    constexpr int BN = 64;
    constexpr int XE = BN * DP;
    __shared__ double xs[XE];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = blockIdx.x * 4 + wave;
    const int n = a.n;
    const int i = tile * 16 + (lane & 15);
    double sc[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) sc[k] = a.scale[k];
    const double sc0sq = sc[0] * sc[0];
    double xi[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) xi[k] = (i < n) ? a.xh[(long long)i * DP + k] : 0.0;

    const int nchunk = a.nchunk;
    const int c0 = (int)(((long long)blockIdx.y * nchunk) / gridDim.y);
    const int c1 = (int)(((long long)(blockIdx.y + 1) * nchunk) / gridDim.y);
    doublex2* __restrict__ out = reinterpret_cast<doublex2*>(static_cast<double*>(a.kt) + (size_t)tile * a.njs * 64) + lane;
    auto entry = [&](int jl) {
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < DP; ++k) {
            const double dd = xi[k] - xs[jl * DP + k];
            if constexpr (ARD) {
                const double u = dd * sc[k];
                r2 = fma(u, u, r2);
            } else {
                r2 = fma(dd, dd, r2);
            }
        }
        if constexpr (!ARD) r2 *= sc0sq;
        return mfma::kentry64<KERNEL>(r2);
    };
    floatx4* __restrict__ out32 = reinterpret_cast<floatx4*>(static_cast<float*>(a.kt) + (size_t)tile * a.njs * 64) + lane;
    // split FP16: a 16-row tile is njs * 16 units of 8 halfs (4 bytes per entry)
    f16x8* __restrict__ out16 = reinterpret_cast<f16x8*>(a.kt) + (size_t)tile * a.njs * 16 + lane;
    for (int c = c0; c < c1; ++c) {
        __syncthreads();
        for (int e = tid; e < XE; e += 256) {
            const int j = c * BN + e / DP;
            xs[e] = (j < n) ? a.xh[(long long)c * BN * DP + e] : 0.0;
        }
        __syncthreads();
        if (ELEM == 2) {
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                f16x8 hv, lv;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const double k = entry(32 * ks + 8 * (lane >> 4) + v);
                    const _Float16 hi = (_Float16)(float)k;
                    hv[v] = hi;
                    lv[v] = (_Float16)(float)((k - (double)hi) * 2048.0);
                }
                __builtin_nontemporal_store(hv, out16 + (size_t)(c * 4 + 2 * ks) * 64);
                __builtin_nontemporal_store(lv, out16 + (size_t)(c * 4 + 2 * ks + 1) * 64);
            }
        } else if (ELEM == 1) {
#pragma unroll 2
            for (int p = 0; p < 4; ++p) {
                floatx4 kv;
#pragma unroll
                for (int h = 0; h < 4; ++h) kv[h] = (float)entry(16 * p + 4 * h + (lane >> 4));
                __builtin_nontemporal_store(kv, out32 + (size_t)(c * 4 + p) * 64);
            }
        } else {
#pragma unroll 2
            for (int p = 0; p < 8; ++p) {
                doublex2 kv;
                kv[0] = entry(8 * p + (lane >> 4));
                kv[1] = entry(8 * p + 4 + (lane >> 4));
                __builtin_nontemporal_store(kv, out + (size_t)(c * 8 + p) * 64);
            }
        }
    }
}

template <int KERNEL, bool ARD, int ELEM>
hipError_t launch_kbuild_dp(const KBuildArgs& a, dim3 grid, hipStream_t st) {
    switch (a.dp) {
        case 4: hipLaunchKernelGGL((kbuild_kernel<KERNEL, 4, ARD, ELEM>), grid, dim3(256), 0, st, a); break;
        case 6: hipLaunchKernelGGL((kbuild_kernel<KERNEL, 6, ARD, ELEM>), grid, dim3(256), 0, st, a); break;
        case 8: hipLaunchKernelGGL((kbuild_kernel<KERNEL, 8, ARD, ELEM>), grid, dim3(256), 0, st, a); break;
        case 10: hipLaunchKernelGGL((kbuild_kernel<KERNEL, 10, ARD, ELEM>), grid, dim3(256), 0, st, a); break;
        case 12: hipLaunchKernelGGL((kbuild_kernel<KERNEL, 12, ARD, ELEM>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((kbuild_kernel<KERNEL, 16, ARD, ELEM>), grid, dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

template <int KERNEL, bool ARD>
hipError_t launch_kbuild_t(const KBuildArgs& a, dim3 grid, hipStream_t st) {
    if (a.elem == 2) return launch_kbuild_dp<KERNEL, ARD, 2>(a, grid, st);
    return a.elem == 1 ? launch_kbuild_dp<KERNEL, ARD, 1>(a, grid, st) : launch_kbuild_dp<KERNEL, ARD, 0>(a, grid, st);
}

// ---- streaming product -----------------------------------------------------
// Y_split = o2 * K[rows, cols(split)] V[cols(split)] (+ s2 V on split 0).
// 1-D grid of nrb * nsplit blocks, split = blockIdx.x % nsplit: consecutive
// blocks go to different XCDs, so with nsplit a multiple of 8 every XCD works
// on one column range and keeps that slice of V in its own L2.
// A block of 4 waves owns 64 * RT rows; wave w owns 16-row tiles
// 4 * RT * rb + RT * w + rt. Per 64-column chunk the rows of V are staged in
// LDS (as in the on-the-fly product) and the wave's 16 * RT operand loads of
// the next chunk are in flight while the current chunk is contracted.
template <int NSB, int RT, int WAVES, int KD>
__global__ __launch_bounds__(64 * WAVES) void mvm_kt_kernel(MvmArgs a) {
    constexpr int NT = 64 * WAVES;
    constexpr int BN = 64;
    constexpr int S16 = NSB * 16;
    constexpr int VST = (NSB & 1) ? S16 : S16 + 16;
    __shared__ __attribute__((aligned(16))) double vs[BN * VST];

    if (mfma::done_now(a.done)) return;
    const int nsplit = a.nsplit;
    const int split = (int)(blockIdx.x % (unsigned)nsplit);
    const int rb = (int)(blockIdx.x / (unsigned)nsplit);
    const int n = a.n;
    const double o2 = a.o2, s2 = a.s2;
    const double* __restrict__ v = static_cast<const double*>(a.v);
    double* __restrict__ y = static_cast<double*>(a.y) + (long long)split * a.ysplit;
    const int s = a.s, ldv = a.ldv, ldy = a.ldy;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: keeps bases in SGPRs
    const int tile0 = (rb * WAVES + wave) * RT;
    const int row0 = tile0 * 16;

    const int nchunk = (n + BN - 1) / BN;
    const int c0 = (int)(((long long)split * nchunk) / nsplit);
    const int c1 = (int)(((long long)(split + 1) * nchunk) / nsplit);

    doublex4 acc[RT][NSB];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) acc[rt][sb] = doublex4{0.0, 0.0, 0.0, 0.0};

    // thread (vr, vc) moves 2 consecutive columns vc*2.. of rows vr + k * VR:
    // one 16-byte load and one 16-byte LDS store each; chunks wholly inside
    // the matrix with every column live and 16-byte aligned rows take the
    // unchecked path
    constexpr int VW = 2;
    using VecT = doublex2;
    constexpr int CW = S16 / VW;
    constexpr int VR = NT / CW;
    constexpr int VPV = BN / VR;
    const int vr = tid / CW, vc = tid - (tid / CW) * CW;
    const bool vec_ok = (s == S16) && (ldv % VW == 0) && ((reinterpret_cast<uintptr_t>(v) & 15) == 0);
    doublex2 vreg[VPV];
    auto fetch_v = [&](int c) {
        const int j0 = c * BN;
        if (vec_ok && j0 + BN <= n) {
#pragma unroll
            for (int k = 0; k < VPV; ++k)
                vreg[k] = *reinterpret_cast<const doublex2*>(v + (size_t)(j0 + vr + k * VR) * ldv + VW * vc);
        } else {
#pragma unroll
            for (int k = 0; k < VPV; ++k) {
                const int j = j0 + vr + k * VR;
#pragma unroll
                for (int h = 0; h < VW; ++h) {
                    const int col = VW * vc + h;
                    vreg[k][h] = (col < s && j < n) ? v[(size_t)j * ldv + col] : 0.0;
                }
            }
        }
    };
    // operand loads: uniform base per (16-row tile, chunk), lane offset l + 64 st
    const double* kb[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) kb[rt] = static_cast<const double*>(a.kt) + (size_t)(tile0 + rt) * a.njs * 64;
    // KD chunks of operands in flight: chunk c + KD - 1 is requested while c
    // is contracted
    double kq[KD][RT][16];
    auto fetch_k = [&](int c, double (&dst)[RT][16]) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const doublex2* base = reinterpret_cast<const doublex2*>(kb[rt] + (size_t)c * 1024);
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const doublex2 x = __builtin_nontemporal_load(base + (unsigned)(lane + 64 * p));
                dst[rt][2 * p] = x[0];
                dst[rt][2 * p + 1] = x[1];
            }
        }
    };
    // one chunk: publish its V rows, start later loads, contract; the B
    // operands of step st + 1 are read from LDS before step st's MFMAs
    auto chunk = [&](int c, double (&cur)[RT][16], double (&far)[RT][16]) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < VPV; ++k) *reinterpret_cast<VecT*>(&vs[(vr + k * VR) * VST + VW * vc]) = vreg[k];
        __syncthreads();
        if (c + 1 < c1) fetch_v(c + 1);
        if (c + KD - 1 < c1) fetch_k(c + KD - 1, far);
        double bcur[NSB], bnxt[NSB];
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) bcur[sb] = vs[(lane >> 4) * VST + sb * 16 + (lane & 15)];
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            if (st + 1 < 16) {
                const int jn = 4 * (st + 1) + (lane >> 4);
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb) bnxt[sb] = vs[jn * VST + sb * 16 + (lane & 15)];
            }
#pragma unroll
            for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    acc[rt][sb] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[rt][st], bcur[sb], acc[rt][sb], 0, 0, 0);
#pragma unroll
            for (int sb = 0; sb < NSB; ++sb) bcur[sb] = bnxt[sb];
        }
    };
    if (c0 < c1) fetch_v(c0);
#pragma unroll
    for (int q = 0; q + 1 < KD; ++q)
        if (c0 + q < c1) fetch_k(c0 + q, kq[q]);
    // KD chunks per trip so the operand buffers rotate without copies
    for (int c = c0; c < c1; c += KD) {
#pragma unroll
        for (int q = 0; q < KD; ++q)
            if (c + q < c1) chunk(c + q, kq[q], kq[(q + KD - 1) % KD]);
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

// FP32 resident matrix (CIQ_F32): the same structure with FP32 operands and
// MFMA, FP32 sums inside a 64-column chunk and FP64 across chunks. The FP32
// sums are the rounding that limits ill-conditioned problems: every product
// adds fresh noise of about 2^-24 |running FP32 sum| per MFMA, which lands
// in the noise-level eigendirections that the inverse root amplifies, and
// it grows as the square root of the MFMA steps B one FP32 sum spans.
// NACC picks B: NACC accumulators take the chunk's 16 steps in rotation
// (B = 16 / NACC, NACC = 1 or 4), and NACC = 0 takes each MFMA's output
// into FP64 at once (B = 1, four converts and adds per MFMA). NACC = -1
// contracts on the FP64 MFMA instead, the FP32 operands converted as they
// are used (two converts per MFMA, no FP32 sums at all): at half the FP32
// MFMA rate, which launches of at most 32 columns can afford, since they
// stream K at HBM speed with the matrix cores less than half busy. Those
// launches use B = 4, or the FP64 MFMA for the inverse root (a.acc); the
// 64-column launch is MFMA-bound and uses B = 16, or B = 4 for the inverse
// root.
// Batched runs (a.wl set) keep one such matrix per problem (a.pkt: its
// element offset, a.pnjs: its padded columns / 4) and run persistently: a
// grid of the resident blocks takes (problem, row block, column range) items
// from the global counter a.queue in list order (largest problem first),
// skipping problems that have stopped.
template <int NSB, int RT, int WAVES, int KD, int NACC>
__device__ __forceinline__ void kt32_item(const MvmArgs& a, int p, int rb, int split, float* vs) {
    constexpr int NT = 64 * WAVES;
    constexpr int BN = 64;
    constexpr int S16 = NSB * 16;
    constexpr int VST = (NSB & 1) ? S16 : S16 + 16;

    const int nsplit = a.nsplit;
    const int n = (p < 0) ? a.n : a.pn[p];
    const long long off = (p < 0) ? 0 : a.poff[p];
    const long long njs = (p < 0) ? a.njs : a.pnjs[p];
    const float* kt = static_cast<const float*>(a.kt) + ((p < 0) ? 0 : a.pkt[p]);
    const double o2 = (p < 0) ? a.o2 : (double)a.po2[p];
    const double s2 = (p < 0) ? a.s2 : (double)a.ps2[p];
    const float* __restrict__ v = static_cast<const float*>(a.v) + off * a.ldv;
    double* __restrict__ y = static_cast<double*>(a.y) + (long long)split * a.ysplit + off * a.ldy;
    float* __restrict__ y32 = a.y32 ? a.y32 + (long long)split * a.ysplit + off * a.ldy : nullptr;
    const int s = a.s, ldv = a.ldv, ldy = a.ldy;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: keeps bases in SGPRs
    const int tile0 = (rb * WAVES + wave) * RT;
    const int row0 = tile0 * 16;

    const int nchunk = (n + BN - 1) / BN;
    const int c0 = (int)(((long long)split * nchunk) / nsplit);
    const int c1 = (int)(((long long)(split + 1) * nchunk) / nsplit);

    // FP32 sums of B = 16 / NACC steps (NACC = 0: one step), FP64 beyond;
    // NACC = -1: FP64 MFMA, in two chains when the wave has one output tile
    static_assert(NACC >= -1 && NACC <= 4 && NACC != 3, "accumulator rotation");
    constexpr bool F64M = NACC < 0;
    constexpr int NA = NACC > 0 ? NACC : 1;
    constexpr int NC = (F64M && RT * NSB == 1) ? 2 : 1;
    floatx4 acc[NA][RT][NSB];
    double accd[RT][NSB][4];
    doublex4 acc64[NC][RT][NSB];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
#pragma unroll
            for (int h = 0; h < NA; ++h) acc[h][rt][sb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) accd[rt][sb][r] = 0.0;
#pragma unroll
            for (int h = 0; h < NC; ++h) acc64[h][rt][sb] = doublex4{0.0, 0.0, 0.0, 0.0};
        }

    // thread (vr, vc) moves 4 consecutive columns vc*4.. of rows vr + k * VR:
    // one 16-byte load and one 16-byte LDS store each; chunks wholly inside
    // the matrix with every column live and 16-byte aligned rows take the
    // unchecked path
    constexpr int VW = 4;
    using VecT = floatx4;
    constexpr int CW = S16 / VW;
    constexpr int VR = NT / CW;
    constexpr int VPV = BN / VR;
    const int vr = tid / CW, vc = tid - (tid / CW) * CW;
    const bool vec_ok = (s == S16) && (ldv % VW == 0) && ((reinterpret_cast<uintptr_t>(v) & 15) == 0);
    floatx4 vreg[VPV];
    auto fetch_v = [&](int c) {
        const int j0 = c * BN;
        if (vec_ok && j0 + BN <= n) {
#pragma unroll
            for (int k = 0; k < VPV; ++k)
                vreg[k] = *reinterpret_cast<const floatx4*>(v + (size_t)(j0 + vr + k * VR) * ldv + VW * vc);
        } else {
#pragma unroll
            for (int k = 0; k < VPV; ++k) {
                const int j = j0 + vr + k * VR;
#pragma unroll
                for (int h = 0; h < VW; ++h) {
                    const int col = VW * vc + h;
                    vreg[k][h] = (col < s && j < n) ? v[(size_t)j * ldv + col] : 0.0f;
                }
            }
        }
    };
    // operand loads: uniform base per (16-row tile, chunk), lane offset l + 64 st
    const float* kb[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) kb[rt] = kt + (size_t)(tile0 + rt) * njs * 64;
    // KD chunks of operands in flight: chunk c + KD - 1 is requested while c
    // is contracted
    float kq[KD][RT][16];
    auto fetch_k = [&](int c, float (&dst)[RT][16]) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const floatx4* base = reinterpret_cast<const floatx4*>(kb[rt] + (size_t)c * 1024);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const floatx4 x = __builtin_nontemporal_load(base + (unsigned)(lane + 64 * p));
#pragma unroll
                for (int h = 0; h < 4; ++h) dst[rt][4 * p + h] = x[h];
            }
        }
    };
    // one chunk: publish its V rows in LDS buffer c % 2, start later loads,
    // contract; the B operands of step st + 1 are read from LDS before step
    // st's MFMAs. One barrier per chunk: a wave writes buffer c % 2 again only
    // after the barrier of chunk c + 1, which every wave reaches after its
    // reads of chunk c (the caller's barrier separates work items).
    auto chunk = [&](int c, float (&cur)[RT][16], float (&far)[RT][16]) {
        float* vb = vs + (c & 1) * (BN * VST);
#pragma unroll
        for (int k = 0; k < VPV; ++k) *reinterpret_cast<VecT*>(&vb[(vr + k * VR) * VST + VW * vc]) = vreg[k];
        __syncthreads();
        if (c + 1 < c1) fetch_v(c + 1);
        if (c + KD - 1 < c1) fetch_k(c + KD - 1, far);
        float bcur[NSB], bnxt[NSB];
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) bcur[sb] = vb[(lane >> 4) * VST + sb * 16 + (lane & 15)];
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            if (st + 1 < 16) {
                const int jn = 4 * (st + 1) + (lane >> 4);
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb) bnxt[sb] = vb[jn * VST + sb * 16 + (lane & 15)];
            }
            if constexpr (F64M) {
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc64[st % NC][rt][sb] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            (double)cur[rt][st], (double)bcur[sb], acc64[st % NC][rt][sb], 0, 0, 0);
            } else if constexpr (NACC == 0) {
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) {
                        const floatx4 t = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            cur[rt][st], bcur[sb], floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
                        for (int r = 0; r < 4; ++r) accd[rt][sb][r] += (double)t[r];
                    }
            } else {
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[st % NA][rt][sb] =
                            __builtin_amdgcn_mfma_f32_16x16x4f32(cur[rt][st], bcur[sb], acc[st % NA][rt][sb], 0, 0, 0);
            }
#pragma unroll
            for (int sb = 0; sb < NSB; ++sb) bcur[sb] = bnxt[sb];
        }
        if constexpr (NACC > 0) {
#pragma unroll
            for (int h = 0; h < NA; ++h)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int sb = 0; sb < NSB; ++sb) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) accd[rt][sb][r] += (double)acc[h][rt][sb][r];
                        acc[h][rt][sb] = floatx4{0.f, 0.f, 0.f, 0.f};
                    }
        }
    };
    if (c0 < c1) fetch_v(c0);
#pragma unroll
    for (int q = 0; q + 1 < KD; ++q)
        if (c0 + q < c1) fetch_k(c0 + q, kq[q]);
    // KD chunks per trip so the operand buffers rotate without copies
    for (int c = c0; c < c1; c += KD) {
#pragma unroll
        for (int q = 0; q < KD; ++q)
            if (c + q < c1) chunk(c + q, kq[q], kq[(q + KD - 1) % KD]);
    }

#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
            const int cc = sb * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // FP32 16x16x4 layout: row 4 (lane / 16) + r; FP64: lane / 16 + 4 r
                const int i = row0 + rt * 16 + (F64M ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
                if (i < n && cc < s) {
                    double sum = accd[rt][sb][r];
                    if constexpr (F64M) {
                        sum = acc64[0][rt][sb][r];
#pragma unroll
                        for (int h = 1; h < NC; ++h) sum += acc64[h][rt][sb][r];
                    }
                    double val = o2 * sum;
                    if (split == 0) val = fma(s2, (double)v[(long long)i * ldv + cc], val);
                    if (y32) y32[(long long)i * ldy + cc] = (float)val;
                    else y[(long long)i * ldy + cc] = val;
                }
            }
        }
    }
}

template <int NSB, int RT, int WAVES, int KD, int NACC>
__global__ __launch_bounds__(64 * WAVES) void mvm_kt32_kernel(MvmArgs a) {
    constexpr int S16 = NSB * 16;
    constexpr int VST = (NSB & 1) ? S16 : S16 + 16;
    __shared__ __attribute__((aligned(16))) float vs[2 * 64 * VST];   // two chunk buffers
    __shared__ int item_sh;
    if (mfma::done_now(a.done)) return;
    if (a.queue != nullptr) {            // batched, persistent
        for (;;) {
            __syncthreads();             // every thread has read the previous item
            if (threadIdx.x == 0) item_sh = atomicAdd(a.queue, 1);
            __syncthreads();
            const int item = item_sh;
            if (item >= a.nitems) break;
            const WorkItem wi = a.wl[item / a.nsplit];
            if (a.prob_done != nullptr && a.prob_done[wi.prob]) continue;
            kt32_item<NSB, RT, WAVES, KD, NACC>(a, wi.prob, wi.rb, item % a.nsplit, vs);
        }
        return;
    }
    kt32_item<NSB, RT, WAVES, KD, NACC>(a, -1, (int)(blockIdx.x / (unsigned)a.nsplit),
                                  (int)(blockIdx.x % (unsigned)a.nsplit), vs);
}

// Split FP16 resident matrix (CIQ_F16X3): the same block structure; per
// 64-column chunk the block stages the chunk's split V operands (NSB column
// blocks x 2 k-steps x hi/lo, already in B-operand order) in LDS with 16-byte
// copies, and each wave contracts its RT tiles' split K operands (four
// 16-byte loads per lane and tile, the next chunk's in flight) with three
// part pairs. For 128-row blocks the wide launches use eight waves of one
// tile each rather than four of two: the V staging is shared by twice the
// rows at 128 VGPRs (four waves per SIMD) instead of 256 (one).
template <int NSB, int RT, int WAVES, int KD>
__global__ __launch_bounds__(64 * WAVES) void mvm_kt16_kernel(MvmArgs a) {
    constexpr int NT = 64 * WAVES;
    constexpr int VU = 2 * NSB * 128;            // 16-byte V units per chunk
    static_assert(VU % NT == 0, "V units per thread");
    constexpr int UPT = VU / NT;
    __shared__ f16x8 vs[2 * VU];   // two chunk buffers (one barrier per chunk, as in kt32_item)

    if (mfma::done_now(a.done)) return;
    const int nsplit = a.nsplit;
    const int split = (int)(blockIdx.x % (unsigned)nsplit);
    const int rb = (int)(blockIdx.x / (unsigned)nsplit);
    const int n = a.n;
    const double o2 = a.o2, s2 = a.s2;
    const double* __restrict__ v = static_cast<const double*>(a.v);
    const f16x8* __restrict__ vt = static_cast<const f16x8*>(a.vt);
    const long long kstride = (long long)a.nsbt * 128;          // units per k-step
    double* __restrict__ y = static_cast<double*>(a.y) + (long long)split * a.ysplit;
    float* __restrict__ y32 = a.y32 ? a.y32 + (long long)split * a.ysplit : nullptr;
    const int s = a.s, ldv = a.ldv, ldy = a.ldy;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tile0 = (rb * WAVES + wave) * RT;
    const int row0 = tile0 * 16;

    const int nchunk = (n + 63) / 64;
    const int c0 = (int)(((long long)split * nchunk) / nsplit);
    const int c1 = (int)(((long long)(split + 1) * nchunk) / nsplit);

    floatx4 ah[RT][NSB], ax[RT][NSB];
    double accd[RT][NSB][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
            ah[rt][sb] = floatx4{0.f, 0.f, 0.f, 0.f};
            ax[rt][sb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) accd[rt][sb][r] = 0.0;
        }

    // unit u of a chunk: k-step kk = u / (NSB * 128) of the chunk, then the
    // NSB column blocks' hi/lo units in buffer order (one contiguous span)
    f16x8 vreg[UPT];
    auto fetch_v = [&](int c) {
#pragma unroll
        for (int m = 0; m < UPT; ++m) {
            const int u = tid + NT * m;
            const int kk = u / (NSB * 128);
            vreg[m] = vt[(long long)(2 * c + kk) * kstride + (u - kk * NSB * 128)];
        }
    };
    const f16x8* kb[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) kb[rt] = static_cast<const f16x8*>(a.kt) + (size_t)(tile0 + rt) * a.njs * 16;
    f16x8 kq[KD][RT][4];
    auto fetch_k = [&](int c, f16x8 (&dst)[RT][4]) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int p = 0; p < 4; ++p)
                dst[rt][p] = __builtin_nontemporal_load(kb[rt] + (size_t)c * 256 + (unsigned)(64 * p + lane));
    };
    auto chunk = [&](int c, f16x8 (&cur)[RT][4], f16x8 (&far)[RT][4]) {
        f16x8* vb = vs + (c & 1) * VU;
#pragma unroll
        for (int m = 0; m < UPT; ++m) vb[tid + NT * m] = vreg[m];
        __syncthreads();
        if (c + 1 < c1) fetch_v(c + 1);
        if (c + KD - 1 < c1) fetch_k(c + KD - 1, far);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
            for (int sb = 0; sb < NSB; ++sb) {
                const f16x8 bh = vb[(kk * NSB + sb) * 128 + lane];
                const f16x8 bl = vb[(kk * NSB + sb) * 128 + 64 + lane];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    ah[rt][sb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(cur[rt][2 * kk], bh, ah[rt][sb], 0, 0, 0);
                    ax[rt][sb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(cur[rt][2 * kk], bl, ax[rt][sb], 0, 0, 0);
                    ax[rt][sb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(cur[rt][2 * kk + 1], bh, ax[rt][sb], 0, 0, 0);
                }
            }
        }
        // the hi x hi sum leaves FP32 after every chunk; the cross sum is
        // 2^-11 smaller and stays in FP32 for the whole range
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int sb = 0; sb < NSB; ++sb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) accd[rt][sb][r] += (double)ah[rt][sb][r];
                ah[rt][sb] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
    };
    if (c0 < c1) fetch_v(c0);
#pragma unroll
    for (int q = 0; q + 1 < KD; ++q)
        if (c0 + q < c1) fetch_k(c0 + q, kq[q]);
    for (int c = c0; c < c1; c += KD) {
#pragma unroll
        for (int q = 0; q < KD; ++q)
            if (c + q < c1) chunk(c + q, kq[q], kq[(q + KD - 1) % KD]);
    }

    constexpr double k11 = 1.0 / 2048.0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
            const int cc = sb * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = row0 + rt * 16 + 4 * (lane >> 4) + r;   // 16x16 accumulator layout
                if (i < n && cc < s) {
                    const double vi = a.vcol_inv ? a.vcol_inv[cc] : a.vinv;
                    const double kv = accd[rt][sb][r] + (double)ax[rt][sb][r] * k11;
                    double val = o2 * kv * vi;
                    if (split == 0) val = fma(s2, v[(long long)i * ldv + cc], val);
                    if (y32) y32[(long long)i * ldy + cc] = (float)val;
                    else y[(long long)i * ldy + cc] = val;
                }
            }
        }
    }
}

template <int NSB>
hipError_t launch_kt_nsb(const MvmArgs& a, int grid, hipStream_t st) {
    if (a.rt == 1)
        hipLaunchKernelGGL((mvm_kt_kernel<NSB, 1, 4, 2>), dim3(grid), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((mvm_kt_kernel<NSB, 2, 4, 2>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace

size_t kcache_rows(int n) { return ((size_t)n + 127) / 128 * 128; }
size_t kcache_cols(int n) { return ((size_t)n + 63) / 64 * 64; }
size_t kcache_bytes(int n, int elem_bytes) { return kcache_rows(n) * kcache_cols(n) * (size_t)elem_bytes; }

hipError_t launch_kbuild(const KBuildArgs& a, hipStream_t st) {
    const int nrb64 = (int)(kcache_rows(a.n) / 64);
    // enough blocks to fill 256 CUs several times over
    int ny = 1;
    while ((long long)nrb64 * ny < 4096 && ny < a.nchunk) ny *= 2;
    dim3 grid(nrb64, ny);
    if (a.kernel == CIQ_KERNEL_RBF)
        return a.ard ? launch_kbuild_t<CIQ_KERNEL_RBF, true>(a, grid, st)
                     : launch_kbuild_t<CIQ_KERNEL_RBF, false>(a, grid, st);
    return a.ard ? launch_kbuild_t<CIQ_KERNEL_MATERN52, true>(a, grid, st)
                 : launch_kbuild_t<CIQ_KERNEL_MATERN52, false>(a, grid, st);
}

template <typename K>
static int occupancy_of(K kernel, int threads = 256) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

// accumulator rotation of a launch (see kt32_item)
constexpr int kt32_nacc(int nsb, int acc) { return nsb <= 2 ? (acc ? -1 : 4) : (acc ? 4 : 1); }

template <int NSB, int RT, int NACC>
hipError_t launch_kt32_variant(const MvmArgs& a, int grid, hipStream_t st) {
    if (a.queue != nullptr) {            // batched: persistent grid of the resident blocks
        static int slots = 0;
        if (slots == 0) {
            int dev = 0, ncu = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
                slots = std::max(1, occupancy_of(mvm_kt32_kernel<NSB, RT, 4, 2, NACC>)) * ncu;
            else
                slots = 1024;
            (void)hipGetLastError();
        }
        const hipError_t e = launch_fill<int>(a.queue, 1, 0, st);
        if (e != hipSuccess) return e;
        grid = std::min(a.nitems, slots);
    }
    hipLaunchKernelGGL((mvm_kt32_kernel<NSB, RT, 4, 2, NACC>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int NSB>
hipError_t launch_kt32_nsb(const MvmArgs& a, int grid, hipStream_t st) {
    constexpr int fast = kt32_nacc(NSB, 0), fine = kt32_nacc(NSB, 1);
    if (a.rt == 1)
        return a.acc ? launch_kt32_variant<NSB, 1, fine>(a, grid, st) : launch_kt32_variant<NSB, 1, fast>(a, grid, st);
    return a.acc ? launch_kt32_variant<NSB, 2, fine>(a, grid, st) : launch_kt32_variant<NSB, 2, fast>(a, grid, st);
}

template <int NSB, int RT>
int kt32_occupancy(int acc) {
    return acc ? occupancy_of(mvm_kt32_kernel<NSB, RT, 4, 2, kt32_nacc(NSB, 1)>)
               : occupancy_of(mvm_kt32_kernel<NSB, RT, 4, 2, kt32_nacc(NSB, 0)>);
}

// the row blocks of a launch must stay inside the padded rows of the matrix
static bool kt_rows_ok(const MvmArgs& a) {
    return a.rt >= 1 && a.rt <= 2 && (size_t)a.nrb * 64 * a.rt <= kcache_rows(a.n) &&
           (size_t)a.nrb * 64 * a.rt >= (size_t)a.n && a.njs * 4 == (long long)kcache_cols(a.n);
}

hipError_t launch_mvm_kt(const MvmArgs& a, int nsb, hipStream_t st) {
    if (!kt_rows_ok(a)) return hipErrorInvalidValue;
    const int grid = a.nrb * a.nsplit;
    switch (nsb) {
        case 1: return launch_kt_nsb<1>(a, grid, st);
        case 2: return launch_kt_nsb<2>(a, grid, st);
        default: return launch_kt_nsb<4>(a, grid, st);
    }
}


// rt = 1: 64-row blocks of four one-tile waves; rt = 2: 128-row blocks, as
// eight one-tile waves (one column block: four two-tile waves)
template <int NSB>
hipError_t launch_kt16_nsb(const MvmArgs& a, int grid, hipStream_t st) {
    if (a.rt == 1 || NSB > 4)
        hipLaunchKernelGGL((mvm_kt16_kernel<NSB, 1, 4, 2>), dim3(grid), dim3(256), 0, st, a);
    else if (NSB == 1)
        hipLaunchKernelGGL((mvm_kt16_kernel<1, 2, 4, 2>), dim3(grid), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((mvm_kt16_kernel<(NSB < 2 ? 2 : NSB), 1, 8, 2>), dim3(grid), dim3(512), 0, st, a);
    return hipGetLastError();
}

int kt_blocks_per_cu(int dtype, int nsb, int rt, int acc) {
    const int k = nsb <= 1 ? 1 : (nsb <= 2 ? 2 : 4);
    if (dtype == CIQ_F16X3) {
        if (nsb > 4) return occupancy_of(mvm_kt16_kernel<8, 1, 4, 2>);
        if (rt == 1)
            return k == 1 ? occupancy_of(mvm_kt16_kernel<1, 1, 4, 2>)
                          : (k == 2 ? occupancy_of(mvm_kt16_kernel<2, 1, 4, 2>) : occupancy_of(mvm_kt16_kernel<4, 1, 4, 2>));
        return k == 1 ? occupancy_of(mvm_kt16_kernel<1, 2, 4, 2>)
                      : (k == 2 ? occupancy_of(mvm_kt16_kernel<2, 1, 8, 2>, 512)
                                : occupancy_of(mvm_kt16_kernel<4, 1, 8, 2>, 512));
    }
    const bool f32 = (dtype == CIQ_F32);
    if (f32) {
        if (rt == 1)
            return k == 1 ? kt32_occupancy<1, 1>(acc) : (k == 2 ? kt32_occupancy<2, 1>(acc) : kt32_occupancy<4, 1>(acc));
        return k == 1 ? kt32_occupancy<1, 2>(acc) : (k == 2 ? kt32_occupancy<2, 2>(acc) : kt32_occupancy<4, 2>(acc));
    }
    if (rt == 1)
        return k == 1 ? occupancy_of(mvm_kt_kernel<1, 1, 4, 2>)
                      : (k == 2 ? occupancy_of(mvm_kt_kernel<2, 1, 4, 2>) : occupancy_of(mvm_kt_kernel<4, 1, 4, 2>));
    return k == 1 ? occupancy_of(mvm_kt_kernel<1, 2, 4, 2>)
                  : (k == 2 ? occupancy_of(mvm_kt_kernel<2, 2, 4, 2>) : occupancy_of(mvm_kt_kernel<4, 2, 4, 2>));
}

hipError_t launch_mvm_kt32(const MvmArgs& a, int nsb, hipStream_t st) {
    if (a.wl == nullptr ? !kt_rows_ok(a) : (a.queue == nullptr || a.pkt == nullptr || a.pnjs == nullptr))
        return hipErrorInvalidValue;
    const int grid = a.nrb * a.nsplit;
    switch (nsb) {
        case 1: return launch_kt32_nsb<1>(a, grid, st);
        case 2: return launch_kt32_nsb<2>(a, grid, st);
        default: return launch_kt32_nsb<4>(a, grid, st);
    }
}

// a.vt points at the launch's first column block; the operand buffer spans
// the matrix's padded columns (k-steps) and nsbt column blocks
hipError_t launch_mvm_kt16(const MvmArgs& a, int nsb, hipStream_t st) {
    if (!kt_rows_ok(a) || a.vt == nullptr || a.nsbt < 1) return hipErrorInvalidValue;
    if (nsb > 4 && a.rt != 1) return hipErrorInvalidValue;
    const int grid = a.nrb * a.nsplit;
    switch (nsb) {
        case 1: return launch_kt16_nsb<1>(a, grid, st);
        case 2: return launch_kt16_nsb<2>(a, grid, st);
        case 3:
        case 4: return launch_kt16_nsb<4>(a, grid, st);
        default: return launch_kt16_nsb<8>(a, grid, st);
    }
}

}  // namespace ciq
