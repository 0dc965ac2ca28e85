// Device kernels of libciq (gfx950).
//
//  * Kernel product Y = o^2 k(X, X) V + sigma^2 V without storing K (Sec. 3.2,
//    Property 1): the MFMA kernels live in mvm_mfma.h (FP32 and FP64 paths);
//    this file holds their dispatch (column groups, split of the j range).
//  * msMINRES step (Appendix C, Alg. S4): one reduction kernel for the six
//    FP64 inner products a Lanczos step needs, one single-block FP64 scalar
//    stage (Lanczos alpha/beta, per-shift Givens QR, stopping rule), and one
//    fused vector update (next Lanczos vector, per-shift search directions,
//    quadrature-weighted solution accumulation).
#include "ciq_internal.h"

#include <cmath>
#include <map>
#include <mutex>
#include <utility>

namespace ciq {

namespace {

}  // namespace

int mvm_rows_per_block(int dtype, int s, int rt) {
    if (dtype == CIQ_F64) return 64 * rt;            // FP64 MFMA: column groups of <= 64
    if (dtype == CIQ_BF16X3 || dtype == CIQ_F16X3) return 64;
    const int nsb = (s > 128 ? 128 : s + 15) / 16;
    return (nsb <= 4 && rt == 2) ? 128 : 64;
}

// Split the j range so the number of equal-cost blocks fills the chip's
// resident slots (256 CUs x blocks resident per CU, set by the kernel's
// register use) with the least idle tail.
int mvm_pick_nsplit(int dtype, int nrb, int n_max, int s) {
    const int cap = (dtype == CIQ_F32) ? 128 : 64;
    const int nsb = (s > cap ? cap : s + 15) / 16;
    const int per_cu = nsb <= 2 ? 4 : 2;
    const int slots = 256 * per_cu;
    const int max_split = 8;
    int best = 1;
    double best_eff = 0.0;
    for (int sp = 1; sp <= max_split; ++sp) {
        const int chunks = (n_max + 63) / 64;
        if (sp > chunks) break;
        const double work = (double)nrb * sp;
        const double rounds = std::ceil(work / slots);
        // efficiency of the last round plus a small per-split cost (partials traffic)
        const double eff = work / (rounds * slots) - 0.02 * (sp - 1);
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = sp;
        }
    }
    return best;
}

hipError_t launch_mvm(int dtype, const MvmArgs& a, hipStream_t st) {
    // Accumulators hold at most 8 (FP32) / 4 (FP64, split forms) column blocks
    // of 16; wider right-hand sides run as column groups, each regenerating its
    // entries.
    // FP32 partials: the resident FP32 and split-FP16 products only
    if (a.y32 != nullptr && !((dtype == CIQ_F32 || dtype == CIQ_F16X3) && a.kt != nullptr && a.wl == nullptr))
        return hipErrorInvalidValue;
    const int cap = product_cap(dtype, a.kt != nullptr);
    for (int c0 = 0; c0 < a.s; c0 += cap) {
        MvmArgs g = a;
        g.s = (a.s - c0 < cap) ? a.s - c0 : cap;
        g.y = static_cast<double*>(a.y) + c0;
        if (a.y32) g.y32 = a.y32 + c0;
        const int nsb = (g.s + 15) / 16;
        hipError_t e;
        if (dtype == CIQ_F16X3 && a.kt != nullptr) {
            g.v = static_cast<const double*>(a.v) + c0;
            g.vt = static_cast<const char*>(a.vt) + (size_t)(c0 / 16) * 128 * 16;   // 128 units of 16 B per block
            if (a.vcol_inv) g.vcol_inv = a.vcol_inv + c0;
            e = launch_mvm_kt16(g, nsb, st);
        } else if (dtype == CIQ_F64 && a.kt != nullptr) {
            g.v = static_cast<const double*>(a.v) + c0;
            e = launch_mvm_kt(g, nsb, st);
        } else if (dtype == CIQ_F32 && a.kt != nullptr) {
            g.v = static_cast<const float*>(a.v) + c0;
            e = launch_mvm_kt32(g, nsb, st);
        } else if (dtype == CIQ_BF16X3 || dtype == CIQ_F16X3) {
            g.v = static_cast<const float*>(a.v) + c0;
            const bool half = (dtype == CIQ_F16X3);
            e = (a.kernel == CIQ_KERNEL_RBF) ? launch_mvm_x3_rbf(g, nsb, a.nrb, half, st)
                                              : launch_mvm_x3_m52(g, nsb, a.nrb, half, st);
        } else if (dtype == CIQ_F64) {
            g.v = static_cast<const double*>(a.v) + c0;
            if (a.kernel == CIQ_KERNEL_RBF)
                e = a.ard ? launch_mvm_f64_rbf_ard(g, nsb, a.nrb, st) : launch_mvm_f64_rbf_iso(g, nsb, a.nrb, st);
            else
                e = a.ard ? launch_mvm_f64_m52_ard(g, nsb, a.nrb, st) : launch_mvm_f64_m52_iso(g, nsb, a.nrb, st);
        } else {
            g.v = static_cast<const float*>(a.v) + c0;
            if (a.kernel == CIQ_KERNEL_RBF)
                e = a.ard ? launch_mvm_f32_rbf_ard(g, nsb, a.nrb, st) : launch_mvm_f32_rbf_iso(g, nsb, a.nrb, st);
            else
                e = a.ard ? launch_mvm_f32_m52_ard(g, nsb, a.nrb, st) : launch_mvm_f32_m52_iso(g, nsb, a.nrb, st);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ----------------------------------------------------------------------------
// Input preparation: xh[i][k] = x[i][k] * scale[k] for k < d, 0 for d <= k < dp.
// ----------------------------------------------------------------------------
struct Scale16 {
    double v[CIQ_MAX_D];
};

template <typename TI>
__global__ void prep_kernel(const TI* x, int n, int d, int dp, Scale16 sc, double* xh) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * dp) return;
    const int i = (int)(e / dp), k = (int)(e - (long long)i * dp);
    xh[e] = (k < d) ? (double)x[(long long)i * d + k] * sc.v[k] : 0.0;
}

template <typename TI>
hipError_t launch_prep(const TI* x, int n, int d, int dp, const double* scale, double* xh, hipStream_t st) {
    Scale16 sc;
    for (int k = 0; k < CIQ_MAX_D; ++k) sc.v[k] = (k < d) ? scale[k] : 0.0;
    const long long total = (long long)n * dp;
    const int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(prep_kernel<TI>, dim3(blocks), dim3(256), 0, st, x, n, d, dp, sc, xh);
    return hipGetLastError();
}
template hipError_t launch_prep<float>(const float*, int, int, int, const double*, double*, hipStream_t);
template hipError_t launch_prep<double>(const double*, int, int, int, const double*, double*, hipStream_t);

// ----------------------------------------------------------------------------
// Sum of split partials: out[i][c] = sum_k ypart[k][i][c].
// ----------------------------------------------------------------------------
template <typename TO>
__global__ void reduce_splits_kernel(const double* ypart, long long ysplit, int nsplit, int ldy, int n,
                                     int s, TO* out, int ldo) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * s) return;
    const int i = (int)(e / s), c = (int)(e - (long long)i * s);
    double acc = ypart[(long long)i * ldy + c];
    for (int k = 1; k < nsplit; ++k) acc += ypart[k * ysplit + (long long)i * ldy + c];
    out[(long long)i * ldo + c] = (TO)acc;
}

template <typename TO>
hipError_t launch_reduce_splits(const double* ypart, long long ysplit, int nsplit, int ldy, int n, int s,
                                TO* out, int ldo, hipStream_t st) {
    const long long total = (long long)n * s;
    hipLaunchKernelGGL(reduce_splits_kernel<TO>, dim3((int)((total + 255) / 256)), dim3(256), 0, st,
                       ypart, ysplit, nsplit, ldy, n, s, out, ldo);
    return hipGetLastError();
}
template hipError_t launch_reduce_splits<float>(const double*, long long, int, int, int, int, float*, int, hipStream_t);
template hipError_t launch_reduce_splits<double>(const double*, long long, int, int, int, int, double*, int, hipStream_t);

// ----------------------------------------------------------------------------
// Lanczos inner products in two passes (classical orthogonalisation, the
// order of Appendix C: v = K q_j - beta_j q_{j-1}; alpha_j = q_j^T v;
// v -= alpha_j q_j; beta_{j+1} = ||v||), FP64 sums of the element products.
//   phase 0: partial sums of q_j . (Y - beta_j q_{j-1})          -> dots[..][0]
//   phase 1: alpha_j = sum of the phase-0 partials (fixed order),
//            partial sums of ||Y - beta_j q_{j-1} - alpha_j q_j||^2 -> dots[..][1]
//   init (phase 1 with q = q_prev = null): ||b||^2.
// Y is the sum of the kernel product's split partials; phase 0 writes that sum
// over the first partial, so phase 1 and the update read one array. Block: TS
// columns x RL row lanes; grid (dots_blocks, ceil(s/TS), nprob); row lanes are
// combined in a fixed order, so the result is deterministic.
// ----------------------------------------------------------------------------
__host__ __device__ inline int col_tile(int s) {
    int ts = 1;
    while (ts < s && ts < 64) ts <<= 1;
    return ts;
}

// Column sum k of the dots partials for global column g, in one fixed order
// everywhere (colsum_kernel, and the consumers when fuse_sums is set): lane r
// of 16 sums blocks r, r + 16, ...; then the 16 lane sums are added in lane
// order. Fused and separate column sums are therefore bitwise equal.
// Lane sum r (of 16): partials of blocks r, r + 16, ... added in that order
// (eight loads issued before their adds).
__device__ inline double colsum_lane(const Dev& d, int k, int g, int r) {
    const int p = g / d.s, c = g - p * d.s;
    const double* base = d.dots + ((long long)p * d.dots_blocks * d.s + c) * 2 + k;
    const long long stride = (long long)d.s * 2;
    double acc = 0.0;
    for (int b0 = r; b0 < d.dots_blocks; b0 += 128) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + 16 * u;
            v[u] = (b < d.dots_blocks) ? base[(long long)b * stride] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (b0 + 16 * u < d.dots_blocks) acc += v[u];
    }
    return acc;
}

// colsum[k * ncol + g] (the fixed order above) for every column, by the whole
// block (nt threads, nt a multiple of 64; sh: nt doubles of LDS): 64 columns
// x nt/64 lanes, each lane computes lane sums r, r + nt/64, ...; the 16 lane
// sums of a column are added in order. The results are
// read by this block after a barrier.
__device__ void block_colsums(const Dev& d, int k, int tid, int nt, double* sh) {
    const int lanes = nt >> 6, cl = tid & 63, ln = tid >> 6;
    for (int g0 = 0; g0 < d.ncol; g0 += 64) {
        const int g = g0 + cl;
        __syncthreads();
        for (int r = ln; r < 16; r += lanes) sh[r * 64 + cl] = (g < d.ncol) ? colsum_lane(d, k, g, r) : 0.0;
        __syncthreads();
        if (ln == 0 && g < d.ncol) {
            double t = 0.0;
            for (int r = 0; r < 16; ++r) t += sh[r * 64 + cl];
            d.colsum[(long long)k * d.ncol + g] = t;
        }
    }
    __syncthreads();
}

__device__ void scalar_stage(const Dev& d, int tid, int nt, int* active_cnt, int& any);

template <typename T>
__global__ __launch_bounds__(256) void dots_kernel(Dev d, T* y, long long ysplit, int nsplit,
                                                   const T* q, const T* qp, int phase,
                                                   const float* __restrict__ y32) {
    __shared__ double sh[256];
    __shared__ double lsum[16 * 64];
    if (d.st->done) return;
    const int TS = col_tile(d.s), RL = 256 / TS;
    const int p = blockIdx.z;
    const int n = d.n[p], off = d.row_off[p], s = d.s;
    const int cl = threadIdx.x % TS, rl = threadIdx.x / TS;
    const int c = blockIdx.y * TS + cl;
    double al = 0.0;
    if (q != nullptr && phase == 1) {
        if (d.fuse_sums & 2) {   // alpha_j of this block's columns from the phase-0 partials
            if (c < s)
                for (int r = rl; r < 16; r += RL) lsum[r * TS + cl] = colsum_lane(d, 0, p * s + c, r);
            __syncthreads();
            if (c < s)
                for (int r = 0; r < 16; ++r) al += lsum[r * TS + cl];
        } else if (c < s) {
            al = d.colsum[p * s + c];
        }
    }
    double acc = 0.0;
    if (c < s) {
        const int g = p * s + c;
        const double bj = (q != nullptr) ? d.beta_cur[g] : 0.0;
        // rows i, i + G, i + 2G, ... (G = gridDim.x * RL) in that order; the
        // split partials of two rows are all requested before they are added
        // (in split order), so their loads are in flight together
        constexpr int U = 2, MS = 16;
        const int G = gridDim.x * RL;
        for (int i0 = blockIdx.x * RL + rl; i0 < n; i0 += U * G) {
            double yv[U];
            if (nsplit <= MS) {
                double part[U][MS];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = i0 + u * G;
                    const long long idx = (long long)(off + i) * s + c;
#pragma unroll
                    for (int k = 0; k < MS; ++k)
                        part[u][k] = (i < n && k < nsplit)
                                         ? (y32 ? (double)y32[k * ysplit + idx] : (double)y[k * ysplit + idx])
                                         : 0.0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    yv[u] = part[u][0];
#pragma unroll
                    for (int k = 1; k < MS; ++k)
                        if (k < nsplit) yv[u] += part[u][k];
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = i0 + u * G;
                    yv[u] = 0.0;
                    if (i < n) {
                        const long long idx = (long long)(off + i) * s + c;
                        yv[u] = (double)y[idx];
                        for (int k = 1; k < nsplit; ++k) yv[u] += (double)y[k * ysplit + idx];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * G;
                if (i >= n) break;
                const long long idx = (long long)(off + i) * s + c;
                if (nsplit > 1 || y32) y[idx] = (T)yv[u];   // the reduced product for phase 1 / update
                if (q == nullptr) {                   // ||b||^2
                    acc = fma(yv[u], yv[u], acc);
                    continue;
                }
                // the same arithmetic, in T, as the update kernel forms q_{j+1} with
                const T vT = (T)yv[u] - (T)bj * qp[idx];
                if (phase == 0) {
                    acc = fma((double)q[idx], (double)vT, acc);
                } else {
                    const double v = (double)(vT - (T)al * q[idx]);
                    acc = fma(v, v, acc);
                }
            }
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < TS && c < s) {
        double sum = 0.0;
        for (int r = 0; r < RL; ++r) sum += sh[r * TS + threadIdx.x];
        d.dots[(((long long)p * d.dots_blocks + blockIdx.x) * s + c) * 2 + (q == nullptr ? 1 : phase)] = sum;
    }
}

// The same two passes for s in {4, 8, 16, 32, 64} with 16-byte loads: lane
// (cg, rl) owns columns 4 cg .. 4 cg + 3 of rows rl, rl + RL, ... (RL = 1024 / s
// rows per block pass), so one load instruction moves 1 KB per wave instead of
// 256 or 512 bytes (the passes are bound by the bytes in flight). Per element
// the arithmetic and the order over the split partials are those of
// dots_kernel; the block partials sum the rows in another order.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
    const dvec2 a = *reinterpret_cast<const dvec2*>(p);
    const dvec2 b = *reinterpret_cast<const dvec2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load4_nt(const double* p, double (&v)[4]) {
    const dvec2 a = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
    const dvec2 b = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p + 2));
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load4_nt(const float* p, float (&v)[4]) {
    const fvec4 a = __builtin_nontemporal_load(reinterpret_cast<const fvec4*>(p));
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// PT: element type of the split partials (phase 0); U: rows per trip
template <typename PT, int U, int phase>
__global__ __launch_bounds__(256) void dots_vec_kernel(Dev d, double* y, const PT* yp, long long ysplit,
                                                       int nsplit, const double* q, const double* qp) {
    __shared__ double sh[256 * 4];
    __shared__ double lsum[16 * 64];
    if (d.st->done) return;
    const int s = d.s, CG = s >> 2, RL = 256 / CG;
    const int p = blockIdx.z;
    const int n = d.n[p], off = d.row_off[p];
    const int cg = threadIdx.x % CG, rl = threadIdx.x / CG;
    const int c = 4 * cg, g = p * s + c;
    double al[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (phase == 1) {
        if (d.fuse_sums & 2) {   // alpha_j from the phase-0 partials, colsum_lane's fixed order
            for (int e = threadIdx.x; e < 16 * s; e += 256) {
                const int r = e / s, col = e - r * s;
                lsum[r * 64 + col] = colsum_lane(d, 0, p * s + col, r);
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 4; ++k)
                for (int r = 0; r < 16; ++r) al[k] += lsum[r * 64 + c + k];
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) al[k] = d.colsum[g + k];
        }
    }
    double bj[4], acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) bj[k] = d.beta_cur[g + k];
    const int G = gridDim.x * RL;
    for (int i0 = blockIdx.x * RL + rl; i0 < n; i0 += U * G) {
        double yv[U][4];
        if constexpr (phase == 0) {
            PT part[U][16][4];   // all of a trip's partials requested before they are added
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * G;
                const long long idx = (long long)(off + i) * s + c;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    if (i < n && k < nsplit) {
                        load4_nt(yp + k * ysplit + idx, part[u][k]);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) part[u][k][e] = (PT)0;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    yv[u][e] = (double)part[u][0][e];
#pragma unroll
                    for (int k = 1; k < 16; ++k)
                        if (k < nsplit) yv[u][e] += (double)part[u][k][e];
                }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * G;
                if (i < n) load4(y + (long long)(off + i) * s + c, yv[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * G;
            if (i >= n) break;
            const long long idx = (long long)(off + i) * s + c;
            if (phase == 0 && (nsplit > 1 || sizeof(PT) == 4)) {   // the reduced product for phase 1 / update
                *reinterpret_cast<dvec2*>(y + idx) = dvec2{yv[u][0], yv[u][1]};
                *reinterpret_cast<dvec2*>(y + idx + 2) = dvec2{yv[u][2], yv[u][3]};
            }
            double qv[4], qpv[4];
            load4(q + idx, qv);
            load4(qp + idx, qpv);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double vT = yv[u][e] - bj[e] * qpv[e];
                if (phase == 0) {
                    acc[e] = fma(qv[e], vT, acc[e]);
                } else {
                    const double v = vT - al[e] * qv[e];
                    acc[e] = fma(v, v, acc[e]);
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) sh[threadIdx.x * 4 + e] = acc[e];
    __syncthreads();
    if (threadIdx.x < s) {
        const int col = threadIdx.x, cgc = col >> 2, e = col & 3;
        double sum = 0.0;
        for (int r = 0; r < RL; ++r) sum += sh[(r * CG + cgc) * 4 + e];
        d.dots[(((long long)p * d.dots_blocks + blockIdx.x) * s + col) * 2 + phase] = sum;
    }
}

// Column sums of the block partials, fixed order: colsum[k * ncol + g] =
// sum_b dots[p][b][c][k]. Block: 64 columns x 16 lanes; lane r sums blocks
// r, r + 16, ... (independent loads in flight), then the 16 lane sums are
// added in lane order.
__global__ __launch_bounds__(1024) void colsum_kernel(Dev d, int k) {
    __shared__ double sh[1024];
    if (d.st->done) return;
    const int cl = threadIdx.x & 63, lane = threadIdx.x >> 6;
    const int g = blockIdx.x * 64 + cl;
    double acc = 0.0;
    if (g < d.ncol) {
        const int p = g / d.s, c = g - p * d.s;
        const double* base = d.dots + ((long long)p * d.dots_blocks * d.s + c) * 2 + k;
        const long long stride = (long long)d.s * 2;
#pragma unroll 8
        for (int b = lane; b < d.dots_blocks; b += 16) acc += base[(long long)b * stride];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (lane == 0 && g < d.ncol) {
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) t += sh[r * 64 + cl];
        d.colsum[(long long)k * d.ncol + g] = t;
    }
}

hipError_t launch_colsum(const Dev& d, int k, hipStream_t st) {
    // the consumers sum the partials themselves: alpha in phase 1 (bit 2),
    // both sums in the scalar stage (bit 1)
    if ((k == 0 && (d.fuse_sums & 2)) || (k == 1 && (d.fuse_sums & 1))) return hipSuccess;
    hipLaunchKernelGGL(colsum_kernel, dim3((d.ncol + 63) / 64), dim3(1024), 0, st, d, k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dots(const Dev& d, T* y, long long ysplit, int nsplit, const T* q, const T* qp,
                       int phase, hipStream_t st, const float* y32) {
    if (y32 != nullptr && (phase != 0 || nsplit > 16)) return hipErrorInvalidValue;
    const bool vec_s = d.s == 4 || d.s == 8 || d.s == 16 || d.s == 32 || d.s == 64;
    if (sizeof(T) == 8 && q != nullptr && qp != nullptr && vec_s && nsplit <= 16 && (phase == 0 || nsplit == 1)) {
        dim3 grid(d.dots_blocks, 1, d.nprob);
        double* yd = reinterpret_cast<double*>(y);
        const double* qd = reinterpret_cast<const double*>(q);
        const double* qpd = reinterpret_cast<const double*>(qp);
        if (phase == 1)
            hipLaunchKernelGGL((dots_vec_kernel<double, 4, 1>), grid, dim3(256), 0, st, d, yd, (const double*)yd,
                               0LL, 1, qd, qpd);
        else if (y32 != nullptr)
            hipLaunchKernelGGL((dots_vec_kernel<float, 1, 0>), grid, dim3(256), 0, st, d, yd, y32, ysplit, nsplit,
                               qd, qpd);
        else
            hipLaunchKernelGGL((dots_vec_kernel<double, 1, 0>), grid, dim3(256), 0, st, d, yd, (const double*)yd,
                               ysplit, nsplit, qd, qpd);
        return hipGetLastError();
    }
    const int TS = col_tile(d.s);
    dim3 grid(d.dots_blocks, (d.s + TS - 1) / TS, d.nprob);
    hipLaunchKernelGGL(dots_kernel<T>, grid, dim3(256), 0, st, d, y, ysplit, nsplit, q, qp, phase, y32);
    return hipGetLastError();
}
template hipError_t launch_dots<double>(const Dev&, double*, long long, int, const double*, const double*, int, hipStream_t,
                                        const float*);

// ----------------------------------------------------------------------------
// Scalar stage (single block, FP64). Initial form: beta_1 = ||b||.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void scalar_init_kernel(Dev d) {
    __shared__ int any;
    __shared__ double sh[1024];
    if (d.fuse_sums & 1) block_colsums(d, 1, threadIdx.x, blockDim.x, sh);
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const int ncol = d.ncol, Q = d.Q;
    for (int g = threadIdx.x; g < ncol; g += blockDim.x) {
        const double b1 = sqrt(d.colsum[ncol + g]);
        const bool ok = (b1 > 0.0) && isfinite(b1);
        d.beta1[g] = ok ? b1 : 0.0;
        d.beta_cur[g] = 0.0;
        d.inv_beta_next[g] = ok ? 1.0 / b1 : 0.0;
        d.colactive[g] = ok ? 1 : 0;
        d.colflag[g] = 0;
        d.col_iters[g] = 0;
        if (ok) any = 1;
        for (int q = 0; q < Q; ++q) {
            const int idx = q * ncol + g;
            d.c1[idx] = 1.0; d.s1[idx] = 0.0; d.c2[idx] = 1.0; d.s2[idx] = 0.0;
            d.phibar[idx] = ok ? b1 : 0.0;
            d.frozen[idx] = ok ? 0 : 1;
            d.relres[idx] = ok ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < d.nprob; p += blockDim.x) {
        int act = 0;
        for (int c = 0; c < d.s; ++c) act |= d.colactive[p * d.s + c];
        d.prob_done[p] = act ? 0 : 1;
    }
    if (threadIdx.x == 0) {
        d.st->iter = 0;
        d.st->live = 0;
        d.st->numeric = 0;
        d.st->done = (any && d.max_iter > 0) ? 0 : 1;
    }
}

hipError_t launch_scalar_init(const Dev& d, hipStream_t st) {
    hipLaunchKernelGGL(scalar_init_kernel, dim3(1), dim3(1024), 0, st, d);
    return hipGetLastError();
}

// One msMINRES iteration's scalar work (Appendix C.2, per shift t_q):
//   alpha_j = q_j^T (K q_j - beta_j q_{j-1})
//   beta_{j+1} = ||K q_j - beta_j q_{j-1} - alpha_j q_j||   (from the two-pass partials)
//   Givens: eps = s_{j-2} beta_j, dhat = c_{j-2} beta_j,
//           delta = c_{j-1} dhat + s_{j-1} (alpha_j + t), gbar = -s_{j-1} dhat + c_{j-1} (alpha_j + t),
//           gamma = hypot(gbar, beta_{j+1}), c = gbar/gamma, s = beta_{j+1}/gamma,
//           tau = c phibar, phibar <- -s phibar
// Stopping: shift frozen at |phibar|/||b|| <= tol; column stops when all its
// shifts are frozen or beta_{j+1} breaks down; run stops at max_iter.
// The body, run by all `nt` threads of one block (active_cnt: nprob ints and
// `any` in that block's LDS); the caller has checked that the run is live and
// colsum holds the column sums of both inner products.
__device__ void scalar_stage(const Dev& d, int tid, int nt, int* active_cnt, int& any) {
    IterState* st = d.st;
    const int ncol = d.ncol, Q = d.Q, s = d.s;
    for (int p = tid; p < d.nprob; p += nt) active_cnt[p] = 0;
    if (tid == 0) any = 0;
    __syncthreads();
    const int iter = st->iter;

    for (int g = tid; g < ncol; g += nt) {
        if (!d.colactive[g]) continue;
        const double bj = d.beta_cur[g];
        double al = d.colsum[g];
        double bn = sqrt(fmax(d.colsum[ncol + g], 0.0));
        // ||K q_j|| ~ sqrt(alpha^2 + beta_j^2 + beta_{j+1}^2) scales the breakdown test
        bool broke = !(bn > d.bd_rtol * sqrt(al * al + bj * bj + bn * bn));
        if (!isfinite(al) || !isfinite(bn)) {
            st->numeric = 1;
            broke = true;
            al = 0.0;
        }
        if (d.bounds_mode) {
            double* tr = d.T + ((long long)iter * ncol + g) * 2;
            tr[0] = al;
            tr[1] = bn;
        }
        d.alpha[g] = al;
        d.beta_next[g] = broke ? 0.0 : bn;
        d.beta_used[g] = bj;
        d.col_iters[g] += 1;
    }
    __syncthreads();

    for (int idx = tid; idx < Q * ncol; idx += nt) {
        const int g = idx % ncol, q = idx / ncol;
        ShiftCoef cf;
        cf.delta = cf.eps = cf.ginv = cf.tau = cf.tauw = 0.0;
        cf.upd = 0;
        cf.pad = 0;
        if (d.colactive[g] && !d.frozen[idx]) {
            const int p = g / s;
            const double a = d.alpha[g] + d.t[p * Q + q];
            const double bj = d.beta_used[g], bn = d.beta_next[g];
            const double c1 = d.c1[idx], s1 = d.s1[idx], c2 = d.c2[idx], s2 = d.s2[idx];
            const double eps = s2 * bj;
            const double dhat = c2 * bj;
            const double delta = c1 * dhat + s1 * a;
            const double gbar = -s1 * dhat + c1 * a;
            const double gamma = hypot(gbar, bn);
            double cn = 1.0, sn = 0.0, ginv = 0.0;
            if (gamma > 0.0 && isfinite(gamma)) {
                cn = gbar / gamma;
                sn = bn / gamma;
                ginv = 1.0 / gamma;
            } else {
                st->numeric = 1;
            }
            const double ph = d.phibar[idx];
            const double tau = cn * ph;
            const double phn = -sn * ph;
            cf.delta = delta;
            cf.eps = eps;
            cf.ginv = ginv;
            cf.tau = tau;
            cf.tauw = d.w[p * Q + q] * tau;
            cf.upd = 1;
            d.c2[idx] = c1; d.s2[idx] = s1; d.c1[idx] = cn; d.s1[idx] = sn;
            d.phibar[idx] = phn;
            const double rr = fabs(phn) / d.beta1[g];
            d.relres[idx] = rr;
            if (rr <= d.tol) d.frozen[idx] = 1;
        }
        d.coef[idx] = cf;
        if (d.clog != nullptr) {
            double* lg = d.clog + ((long long)iter * Q * ncol + idx) * 4;
            lg[0] = cf.delta;
            lg[1] = cf.eps;
            lg[2] = cf.ginv;
            lg[3] = cf.tauw;
        }
    }
    __syncthreads();

    for (int g = tid; g < ncol; g += nt) {
        if (!d.colactive[g]) {
            d.colflag[g] = 0;
            continue;
        }
        const bool broke = (d.beta_next[g] == 0.0);
        bool all_frozen = (Q > 0);
        for (int q = 0; q < Q; ++q) all_frozen = all_frozen && d.frozen[q * ncol + g];
        const bool cont = !(broke || all_frozen);
        d.colflag[g] = cont ? 2 : 1;
        d.inv_beta_next[g] = cont ? 1.0 / d.beta_next[g] : 0.0;
        if (cont) {
            d.beta_cur[g] = d.beta_next[g];
            atomicAdd(&active_cnt[g / s], 1);
            any = 1;
        } else {
            d.colactive[g] = 0;
            for (int q = 0; q < Q; ++q) d.frozen[q * ncol + g] = 1;
        }
    }
    __syncthreads();
    for (int p = tid; p < d.nprob; p += nt) d.prob_done[p] = active_cnt[p] ? 0 : 1;
    if (tid == 0) {
        st->iter = iter + 1;
        st->live = 1;
        if (!any || iter + 1 >= d.max_iter) st->done = 1;
    }
}

__global__ __launch_bounds__(1024) void scalar_kernel(Dev d) {
    __shared__ int active_cnt[1024];
    __shared__ int any;
    __shared__ double sh[1024];
    if (d.st->done) {
        if (threadIdx.x == 0) d.st->live = 0;
        return;
    }
    if (d.fuse_sums & 1) {  // column sums of both inner products' partials
        block_colsums(d, 0, threadIdx.x, blockDim.x, sh);
        block_colsums(d, 1, threadIdx.x, blockDim.x, sh);
    }
    scalar_stage(d, threadIdx.x, blockDim.x, active_cnt, any);
}

hipError_t launch_scalar(const Dev& d, hipStream_t st) {
    hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(1024), 0, st, d);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Fused vector update of one msMINRES iteration (column g, row i):
//   per unfrozen shift q: m_j = (q_j - delta m_{j-1} - eps m_{j-2}) * ginv,
//                          acc += w_q tau m_j,  x^{(q)} += tau m_j  (if kept)
//   if the column continues: q_{j+1} = (K q_j - beta_j q_{j-1} - alpha_j q_j) / beta_{j+1}
// (preconditioned form, Appendix D: the recurrence consumes p_j = P^{-1} z_j
// and the continuing column scales the finished w and P^{-1} w, see launch_update)
// m_j overwrites m_{j-2}; q_{j+1} overwrites q_{j-1}.
// Block: TS columns x RL row lanes; grid (blocks, ceil(s/TS), nprob).
// ----------------------------------------------------------------------------
// Element (i, c) of the split FP16 operand copy (op16_index layout), x scaled
// by `scale` first (a power of two, so the split is of x itself).
__device__ inline void put_op16(_Float16* vt, int nsbt, int i, int c, double x, float scale) {
    const double xs = x * (double)scale;
    const _Float16 hi = (_Float16)(float)xs;
    const _Float16 lo = (_Float16)(float)((xs - (double)hi) * 2048.0);
    const size_t k = op16_index(i, c, nsbt);
    vt[k] = hi;
    vt[k + 512] = lo;
}

template <typename T>
__global__ __launch_bounds__(256) void update_kernel(Dev d, const T* y, long long ysplit, int nsplit,
                                                     const T* qcur, T* qprev, const T* m_prev,
                                                     T* m_cur, T* acc, T* solves, long long mstride,
                                                     int TS, float* q32, T* pnext, Op16 op) {
    extern __shared__ char smem[];
    if (!d.st->live) return;
    const int RL = 256 / TS;
    const int s = d.s, ncol = d.ncol;
    // resident basis: no per-shift directions move; q_{j+1} goes to slot j
    const bool basis = d.basis != nullptr;
    const int Q = basis ? 0 : d.Q;
    const int slot = d.st->iter;
    double* const bq = (basis && slot < d.basis_slots) ? d.basis[slot] : nullptr;
    T* sdelta = reinterpret_cast<T*>(smem);
    T* seps = sdelta + Q * TS;
    T* sginv = seps + Q * TS;
    T* stau = sginv + Q * TS;
    T* stauw = stau + Q * TS;
    int* supd = reinterpret_cast<int*>(stauw + Q * TS);
    const int p = blockIdx.z;
    const int cbase = blockIdx.y * TS;
    for (int e = threadIdx.x; e < Q * TS; e += blockDim.x) {
        const int q = e / TS, cc = e % TS;
        const int c = cbase + cc;
        ShiftCoef cf;
        if (c < s) {
            cf = d.coef[q * ncol + p * s + c];
        } else {
            cf.delta = cf.eps = cf.ginv = cf.tau = cf.tauw = 0.0;
            cf.upd = 0;
        }
        sdelta[e] = (T)cf.delta; seps[e] = (T)cf.eps; sginv[e] = (T)cf.ginv;
        stau[e] = (T)cf.tau; stauw[e] = (T)cf.tauw; supd[e] = cf.upd;
    }
    __syncthreads();
    const int cl = threadIdx.x % TS, rl = threadIdx.x / TS;
    const int c = cbase + cl;
    if (c >= s) return;
    const int g = p * s + c;
    const int flag = d.colflag[g];
    if (flag == 0) return;
    const int n = d.n[p], off = d.row_off[p];
    const T al = (T)d.alpha[g];
    const T bj = (T)d.beta_used[g];
    const T ib = (T)d.inv_beta_next[g];
    for (int i = blockIdx.x * RL + rl; i < n; i += gridDim.x * RL) {
        const long long row = off + i;
        const long long idx = row * s + c;
        const T qj = qcur[idx];
        T a = (T)0;
        for (int q = 0; q < Q; ++q) {
            const int e = q * TS + cl;
            if (!supd[e]) continue;
            const long long midx = q * mstride + idx;
            const T m = (qj - sdelta[e] * m_prev[midx] - seps[e] * m_cur[midx]) * sginv[e];
            m_cur[midx] = m;
            a += stauw[e] * m;
            if (solves) solves[(row * Q + q) * s + c] += stau[e] * m;
        }
        if (!basis) acc[idx] += a;
        if (flag == 2) {
            if (pnext) {                        // preconditioned: y is w = z_{j+1} beta_{j+1}
                qprev[idx] = y[idx] * ib;
                const T pn = pnext[idx] * ib;
                pnext[idx] = pn;
                if (q32) q32[idx] = (float)pn;
                else if (op.p) put_op16(static_cast<_Float16*>(op.p), op.nsbt, i, c, (double)pn, op.scale);
                continue;
            }
            double ys = (double)y[idx];
            for (int k = 1; k < nsplit; ++k) ys += (double)y[k * ysplit + idx];
            const T vT = (T)ys - bj * qprev[idx];     // same arithmetic as the inner products
            const T v = vT - al * qj;
            const T qn = v * ib;
            qprev[idx] = qn;
            if (bq) bq[idx] = (double)qn;
            if (q32) q32[idx] = (float)qn;      // operand copy for the FP32 kernel product
            else if (op.p) put_op16(static_cast<_Float16*>(op.p), op.nsbt, i, c, (double)qn, op.scale);
        }
    }
}

// Blocks of update_kernel<T> with shm bytes of coefficient tile that the
// current device holds at once (512 if the runtime cannot say), per
// (device, tile size), cached: the launch comes once per iteration.
template <typename T>
static int update_resident_blocks(size_t shm) {
    static std::mutex mu;
    static std::map<std::pair<int, size_t>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 512;
    }
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, shm});
    if (it != cache.end()) return it->second;
    int per_cu = 0, ncu = 0;
    int blocks = 512;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, update_kernel<T>, 256, shm) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0 &&
        ncu > 0)
        blocks = per_cu * ncu;
    else
        (void)hipGetLastError();
    cache[{dev, shm}] = blocks;
    return blocks;
}

template <typename T>
hipError_t launch_update(const Dev& d, const T* y, long long ysplit, int nsplit, const T* qcur, T* qprev,
                         const T* m_prev, T* m_cur, T* acc, T* solves, float* q32, int max_n, hipStream_t st,
                         T* pnext, Op16 op) {
    const size_t per = 5 * sizeof(T) + sizeof(int);   // LDS bytes per (shift, column)
    int TS = col_tile(d.s);
    while (TS > 1 && (size_t)d.Q * TS * per > 49152) TS >>= 1;   // coefficient tile <= 48 KB LDS
    const int RL = 256 / TS;
    const size_t shm = (size_t)d.Q * TS * per;
    // as many row blocks as the device holds at once with this coefficient
    // tile (the kernel strides over the rest of the rows)
    int bx = (max_n + RL - 1) / RL;
    const int cap = update_resident_blocks<T>(shm);
    if (bx > cap) bx = cap;
    if (bx < 1) bx = 1;
    dim3 grid(bx, (d.s + TS - 1) / TS, d.nprob);
    const long long mstride = (long long)d.rows_total * d.s;
    hipLaunchKernelGGL(update_kernel<T>, grid, dim3(256), shm, st, d, y, ysplit, nsplit, qcur, qprev,
                       m_prev, m_cur, acc, solves, mstride, TS, q32, pnext, op);
    return hipGetLastError();
}
template hipError_t launch_update<double>(const Dev&, const double*, long long, int, const double*, double*,
                                          const double*, double*, double*, double*, float*, int, hipStream_t,
                                          double*, Op16);

// ----------------------------------------------------------------------------
// Resident-basis combine. Per shift and column the logged coefficients give
// the direction recurrence m_j = (q_j - delta_j m_{j-1} - eps_j m_{j-2}) ginv_j
// and the weighted solution x = sum_j tauw_j m_j; expanding the highest m_j
// first, x = sum_j c_j q_j with c_j = a_j ginv_j, where a_j = tauw_j plus what
// the later terms pass down (-c_{j+1} delta_{j+1}, -c_{j+2} eps_{j+2}). A
// frozen shift logs zeros from its freeze on, a stopped column stops at its
// own iteration count, so both truncate the sums exactly as the recurrence
// stops moving them.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void basis_coef_kernel(Dev d, int iters, double* __restrict__ cq) {
    const int QN = d.Q * d.ncol;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= QN) return;
    const int g = idx % d.ncol;
    const int J = min(d.col_iters[g], iters);
    const double* __restrict__ log = d.clog;
    double r1 = 0.0, r2 = 0.0;
    for (int j = J; j >= 1; --j) {
        const double* lg = log + ((long long)(j - 1) * QN + idx) * 4;
        const double c = (lg[3] + r1) * lg[2];
        cq[(long long)(j - 1) * QN + idx] = c;
        r1 = r2 - c * lg[0];
        r2 = -c * lg[1];
    }
}

// c[j][g] = sum over shifts of cq[j][q][g] (in shift order); 0 past the column's run
__global__ __launch_bounds__(256) void basis_csum_kernel(Dev d, int iters, const double* __restrict__ cq,
                                                         double* __restrict__ c) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)iters * d.ncol) return;
    const int j = (int)(e / d.ncol), g = (int)(e - (long long)j * d.ncol);
    double t = 0.0;
    if (j < d.col_iters[g]) {
        const double* row = cq + (long long)j * d.Q * d.ncol + g;
        for (int q = 0; q < d.Q; ++q) t += row[(long long)q * d.ncol];
    }
    c[e] = t;
}

// acc[i][c] = sum_j c[j][g] q_{j+1}[i][c] (slot j, through the slot table),
// j ascending; eight slots' loads in flight per step
__global__ __launch_bounds__(256) void basis_gemv_kernel(Dev d, const double* __restrict__ c,
                                                         double* __restrict__ acc) {
    const int p = blockIdx.z;
    const int n = d.n[p], off = d.row_off[p], s = d.s;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * s) return;
    const int i = (int)(e / s), cc = (int)(e - (long long)i * s);
    const int g = p * s + cc;
    const long long idx = (long long)(off + i) * s + cc;
    const int J = min(d.col_iters[g], d.basis_slots);
    double* const* __restrict__ tab = d.basis;
    const double* __restrict__ cg = c + g;
    const long long cs = d.ncol;
    double t = 0.0;
    int j = 0;
    for (; j + 8 <= J; j += 8) {
        double v[8], w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            v[u] = __builtin_nontemporal_load(tab[j + u] + idx);
            w[u] = cg[(long long)(j + u) * cs];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) t = fma(w[u], v[u], t);
    }
    for (; j < J; ++j) t = fma(cg[(long long)j * cs], tab[j][idx], t);
    acc[idx] = t;
}

// tab[t] for slots t in [first, end): slot t sits at byte offset
// (t % per_chunk) * stride of chunk t / per_chunk, whose base is
// c.base[t / per_chunk - k0] (every slot of the range lies in chunks
// k0 .. k0 + kBasisChunksPerLaunch - 1)
__global__ __launch_bounds__(256) void basis_table_kernel(double** __restrict__ tab, int first, int end,
                                                          int per_chunk, long long stride, int k0, BasisChunks c) {
    const int t = first + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= end) return;
    const int k = t / per_chunk;
    tab[t] = reinterpret_cast<double*>(c.base[k - k0] + (long long)(t - k * per_chunk) * stride);
}

hipError_t launch_basis_table(double** tab, int first, int end, int per_chunk, size_t stride, int k0,
                              const BasisChunks& c, hipStream_t st) {
    if (end <= first) return hipSuccess;
    if (first / per_chunk < k0 || (end - 1) / per_chunk >= k0 + kBasisChunksPerLaunch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(basis_table_kernel, dim3((unsigned)((end - first + 255) / 256)), dim3(256), 0, st, tab, first,
                       end, per_chunk, (long long)stride, k0, c);
    return hipGetLastError();
}

hipError_t launch_basis_combine(const Dev& d, int iters, double* cq, double* c, double* acc, int max_n,
                                hipStream_t st) {
    if (iters <= 0 || d.basis == nullptr || d.clog == nullptr) return hipErrorInvalidValue;
    const int QN = d.Q * d.ncol;
    hipLaunchKernelGGL(basis_coef_kernel, dim3((QN + 255) / 256), dim3(256), 0, st, d, iters, cq);
    const long long ce = (long long)iters * d.ncol;
    hipLaunchKernelGGL(basis_csum_kernel, dim3((unsigned)((ce + 255) / 256)), dim3(256), 0, st, d, iters, cq, c);
    const long long ge = (long long)max_n * d.s;
    hipLaunchKernelGGL(basis_gemv_kernel, dim3((unsigned)((ge + 255) / 256), 1, d.nprob), dim3(256), 0, st, d, c,
                       acc);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Start of a run: q_1 = b / ||b|| (0 for a zero column), q_0 = 0, acc = 0.
// The caller has copied B into q and zeroed the direction/solve buffers.
// ----------------------------------------------------------------------------
template <typename T>
__global__ void init_vectors_kernel(Dev d, T* q, T* qprev, T* acc, float* q32, T* pvec, Op16 op) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)d.rows_total * d.s;
    if (e >= total) return;
    const int row = (int)(e / d.s), c = (int)(e - (long long)row * d.s);
    int p = 0;
    while (p + 1 < d.nprob && d.row_off[p + 1] <= row) ++p;
    const T inv = (T)d.inv_beta_next[p * d.s + c];
    const T qv = q[e] * inv;
    q[e] = qv;
    if (pvec) {
        const T pv = pvec[e] * inv;
        pvec[e] = pv;
        if (q32) q32[e] = (float)pv;
        else if (op.p) put_op16(static_cast<_Float16*>(op.p), op.nsbt, row, c, (double)pv, op.scale);
    } else if (q32) {
        q32[e] = (float)qv;
    } else if (op.p) {
        put_op16(static_cast<_Float16*>(op.p), op.nsbt, row, c, (double)qv, op.scale);
    }
    qprev[e] = (T)0;
    acc[e] = (T)0;
}

template <typename T>
hipError_t launch_init_vectors(const Dev& d, T* q, T* qprev, T* acc, float* q32, int rows, hipStream_t st,
                               T* pvec, Op16 op) {
    const long long total = (long long)rows * d.s;
    hipLaunchKernelGGL(init_vectors_kernel<T>, dim3((int)((total + 255) / 256)), dim3(256), 0, st, d, q,
                       qprev, acc, q32, pvec, op);
    return hipGetLastError();
}
template hipError_t launch_init_vectors<double>(const Dev&, double*, double*, double*, float*, int, hipStream_t,
                                                double*, Op16);

// ----------------------------------------------------------------------------
// Split FP16 operand of an arbitrary FP64 block vector: per column a power of
// two 2^e with max_i |x[i][c]| 2^e in [128, 256) (1 for a zero column), then
// the op16 split of x[i][c] 2^e. inv[c] = 2^-e undoes it in the product.
// Block: 64 columns x 16 row lanes, fixed combination order.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void op16_scale_kernel(const double* x, int n, int s, int ld, double* scale,
                                                          double* inv) {
    __shared__ double sh[1024];
    const int cl = threadIdx.x & 63, lane = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl;
    double m = 0.0;
    if (c < s)
        for (int i = lane; i < n; i += 16) m = fmax(m, fabs(x[(long long)i * ld + c]));
    sh[threadIdx.x] = m;
    __syncthreads();
    if (lane == 0 && c < s) {
        for (int r = 1; r < 16; ++r) m = fmax(m, sh[r * 64 + cl]);
        double sc = 1.0;
        if (m > 0.0 && isfinite(m)) {
            int e = 0;
            (void)frexp(m, &e);          // m in [2^(e-1), 2^e)
            sc = ldexp(1.0, 8 - e);      // m sc in [128, 256)
        }
        scale[c] = sc;
        inv[c] = 1.0 / sc;
    }
}

__global__ void op16_split_kernel(const double* x, int n, int s, int ld, const double* scale, _Float16* vt,
                                  int nsbt) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * s) return;
    const int i = (int)(e / s), c = (int)(e - (long long)i * s);
    put_op16(vt, nsbt, i, c, x[(long long)i * ld + c], (float)scale[c]);
}

hipError_t launch_op16_split(const double* x, int n, int s, int ld, double* scale, double* inv, void* vt,
                             int nsbt, hipStream_t st) {
    hipLaunchKernelGGL(op16_scale_kernel, dim3((s + 63) / 64), dim3(1024), 0, st, x, n, s, ld, scale, inv);
    const long long total = (long long)n * s;
    hipLaunchKernelGGL(op16_split_kernel, dim3((int)((total + 255) / 256)), dim3(256), 0, st, x, n, s, ld, scale,
                       static_cast<_Float16*>(vt), nsbt);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Strided copy, fill, counter-based random start vector.
// ----------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ void copy2d_kernel(const TI* src, int ld_src, int n, int s, TO* dst, int ld_dst) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * s) return;
    const int i = (int)(e / s), c = (int)(e - (long long)i * s);
    dst[(long long)i * ld_dst + c] = (TO)src[(long long)i * ld_src + c];
}

template <typename TI, typename TO>
hipError_t launch_copy(const TI* src, int ld_src, int n, int s, TO* dst, int ld_dst, hipStream_t st) {
    const long long total = (long long)n * s;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL((copy2d_kernel<TI, TO>), dim3((int)((total + 255) / 256)), dim3(256), 0, st, src,
                       ld_src, n, s, dst, ld_dst);
    return hipGetLastError();
}
template hipError_t launch_copy<float, float>(const float*, int, int, int, float*, int, hipStream_t);
template hipError_t launch_copy<double, double>(const double*, int, int, int, double*, int, hipStream_t);
template hipError_t launch_copy<float, double>(const float*, int, int, int, double*, int, hipStream_t);
template hipError_t launch_copy<double, float>(const double*, int, int, int, float*, int, hipStream_t);

template <typename T>
__global__ void fill_kernel(T* p, size_t count, T value) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = value;
}

template <typename T>
hipError_t launch_fill(T* p, size_t count, T value, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count,
                       value);
    return hipGetLastError();
}
template hipError_t launch_fill<float>(float*, size_t, float, hipStream_t);
template hipError_t launch_fill<double>(double*, size_t, double, hipStream_t);
template hipError_t launch_fill<int>(int*, size_t, int, hipStream_t);

// SplitMix64 (Steele, Lea, Flood 2014) evaluated at counter i: a uniform
// draw on [-1, 1) per entry, independent of the launch shape.
__device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ void splitmix_kernel(T* v, int n, uint64_t seed, int ld) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t z = splitmix64(seed + 0x9E3779B97F4A7C15ull * (uint64_t)i);
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    v[(long long)i * ld] = (T)(2.0 * u - 1.0);
}

template <typename T>
hipError_t launch_splitmix(T* v, int n, uint64_t seed, int ld, hipStream_t st) {
    hipLaunchKernelGGL(splitmix_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, v, n, seed, ld);
    return hipGetLastError();
}
template hipError_t launch_splitmix<float>(float*, int, uint64_t, int, hipStream_t);
template hipError_t launch_splitmix<double>(double*, int, uint64_t, int, hipStream_t);

}  // namespace ciq
