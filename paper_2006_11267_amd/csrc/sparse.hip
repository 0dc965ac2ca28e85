// Products with a caller-supplied sparse symmetric operator (CSR, FP64): the
// structured-operator form of msMINRES-CIQ (Sec. 5.3 applies it to the
// precision of an image model). The Krylov machinery is unchanged; only the
// product is this kernel instead of the kernel-matrix product.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ciq_internal.h"

namespace ciq {

namespace {

// Structure check of a caller's CSR operator before any product reads it:
// row_ptr[0] = 0, row_ptr non-decreasing, row_ptr[n] = nnz and every column
// index in [0, n). Reads only row_ptr[0..n] and col[0..nnz); sets *bad on a
// violation.
__global__ void csr_check_kernel(const int* __restrict__ row_ptr, const int* __restrict__ col, int n, int nnz,
                                 int* bad) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long i = t; i <= n; i += stride) {
        const int r = row_ptr[i];
        if ((i == 0 && r != 0) || (i == n && r != nnz) || (i < n && row_ptr[i + 1] < r)) atomicOr(bad, 1);
    }
    for (long long k = t; k < nnz; k += stride) {
        const int c = col[k];
        if (c < 0 || c >= n) atomicOr(bad, 1);
    }
}

// y[i][c] = sum_k val[k] x[col[k]][c] over row i's entries (s > 1). Block: TS columns
// x RL rows (TS = the power of two >= s, at most 64); each thread one (row,
// column), entries in storage order (deterministic).
__global__ __launch_bounds__(256) void spmv_kernel(SparseOp a, const double* __restrict__ x, int ldx, int s,
                                                   double* __restrict__ y, int ldy, int TS, const int* done) {
    if (done != nullptr && *done) return;
    const int RL = 256 / TS;
    const int cl = threadIdx.x % TS, rl = threadIdx.x / TS;
    const int row = blockIdx.x * RL + rl, c = blockIdx.y * TS + cl;
    if (row >= a.n || c >= s) return;
    double acc = 0.0;
    const int k1 = a.row_ptr[row + 1];
    for (int k = a.row_ptr[row]; k < k1; ++k) acc = fma(a.val[k], x[(long long)a.col[k] * ldx + c], acc);
    y[(long long)row * ldy + c] = acc;
}

// One column (s = 1): 16 lanes per row, lane g takes the row's entries
// g, g + 16, ... (coalesced loads of val and col across the 16 lanes), the
// 16 partial sums are combined by a fixed butterfly (deterministic).
__global__ __launch_bounds__(256) void spmv1_kernel(SparseOp a, const double* __restrict__ x,
                                                    double* __restrict__ y, const int* done) {
    if (done != nullptr && *done) return;
    const int g = threadIdx.x & 15;
    const int row = blockIdx.x * 16 + (threadIdx.x >> 4);
    double acc = 0.0;
    if (row < a.n) {
        const int k1 = a.row_ptr[row + 1];
        for (int k = a.row_ptr[row] + g; k < k1; k += 16) acc = fma(a.val[k], x[a.col[k]], acc);
    }
#pragma unroll
    for (int m = 8; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 16);
    if (row < a.n && g == 0) y[row] = acc;
}

}  // namespace

hipError_t launch_csr_check(const int* row_ptr, const int* col, int n, int nnz, int* bad, hipStream_t st) {
    const long long work = std::max((long long)n + 1, (long long)nnz);
    const int blocks = (int)std::min<long long>((work + 255) / 256, 4096);
    hipLaunchKernelGGL(csr_check_kernel, dim3(blocks), dim3(256), 0, st, row_ptr, col, n, nnz, bad);
    return hipGetLastError();
}

hipError_t launch_spmv(const SparseOp& a, const double* x, int ldx, int s, double* y, int ldy, const int* done,
                       hipStream_t st) {
    if (s == 1 && ldx == 1 && ldy == 1) {
        hipLaunchKernelGGL(spmv1_kernel, dim3((a.n + 15) / 16), dim3(256), 0, st, a, x, y, done);
        return hipGetLastError();
    }
    int TS = 1;
    while (TS < s && TS < 64) TS <<= 1;
    const int RL = 256 / TS;
    dim3 grid((a.n + RL - 1) / RL, (s + TS - 1) / TS);
    hipLaunchKernelGGL(spmv_kernel, grid, dim3(256), 0, st, a, x, ldx, s, y, ldy, TS, done);
    return hipGetLastError();
}

}  // namespace ciq
