// Host driver and C ABI of libciq.
//
// One solver call: validate -> (optional) allocate and build the resident
// kernel matrix -> scale/pad points on the device -> (optional) Lanczos
// extreme-eigenvalue estimate -> HHT shifts/weights on the host -> msMINRES
// loop (per iteration: kernel product, two-pass Lanczos inner products,
// scalar Givens stage, fused vector update; all queued on the caller's
// stream, optionally replayed from a HIP graph; the host polls a device
// "done" flag every few iterations) -> combine.
#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <tuple>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "ciq.h"
#include "basis_slots.h"
#include "ciq_internal.h"

namespace ciq {
int hht_quadrature(double lmin, double lmax, int Q, double* t, double* w);
void bounds_from_tridiag(int J, const double* alpha, const double* beta, double noise, double* lmin,
                         double* lmax);
void sym_eig_tridiag(int n, std::vector<double>& a, std::vector<double>& evals, std::vector<double>& v);
}  // namespace ciq

using namespace ciq;

namespace {

constexpr int kMaxDevices = 64;
constexpr double kSqrt5 = 2.23606797749978969640917366873;

#define HIPCHK(expr)                        \
    do {                                    \
        hipError_t e_ = (expr);             \
        if (e_ != hipSuccess) return CIQ_EHIP; \
    } while (0)

#define STCHK(expr)                 \
    do {                            \
        int s_ = (expr);            \
        if (s_ != CIQ_OK) return s_; \
    } while (0)

// ---- per-device grow-only scratch ---------------------------------------
struct DeviceScratch {
    void* ptr = nullptr;
    size_t cap = 0;
    IterState* pinned = nullptr;  // host-pinned mirror of the iteration state
    std::mutex mu;
};
DeviceScratch g_scratch[kMaxDevices];

// ---- Krylov basis chunks kept between calls ---------------------------------
// The resident basis takes up to max_iter + 1 vectors of rows_total * s
// doubles (154 GB at N = 50,000, s = 64, 6000 iterations). Freeing a block
// of tens of GB and allocating the next has been measured to take about two
// seconds each on some driver states, so the slots live in fixed-size chunks
// that stay allocated on the device after a call; the next call reuses them,
// and a run takes new chunks only as its iteration count reaches them (the
// memory held is what the longest run used). The coefficient logs of the
// combine live in one grow-only buffer beside them. Guarded by the device's
// scratch lock; ciq_release_workspace returns all of it.
struct BasisPool {
    std::vector<void*> chunks;
    size_t chunk_bytes = 0;
    void* logs = nullptr;
    size_t logs_cap = 0;
};
BasisPool g_basis[kMaxDevices];

// Frees the pool of the current device `dev` (after the device drains).
int basis_pool_release(int dev) {
    BasisPool& bp = g_basis[dev];
    if (bp.chunks.empty() && !bp.logs) return CIQ_OK;
    HIPCHK(hipDeviceSynchronize());
    hipError_t e = hipSuccess;
    for (void* c : bp.chunks) {
        const hipError_t f = hipFree(c);
        if (f != hipSuccess) e = f;
    }
    bp.chunks.clear();
    if (bp.logs) {
        const hipError_t f = hipFree(bp.logs);
        if (f != hipSuccess) e = f;
    }
    bp.logs = nullptr;
    bp.logs_cap = 0;
    HIPCHK(e);
    return CIQ_OK;
}

// hipMalloc on the current device; when the device is short it first returns
// the basis chunks kept from earlier calls and tries once more. `locked`: the
// caller holds the device's scratch lock; otherwise the lock is taken here
// for the release (a solve running on another thread finishes first).
bool dev_malloc(void** p, size_t bytes, bool locked = true) {
    if (hipMalloc(p, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    *p = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return false;
    }
    std::unique_lock<std::mutex> lk(g_scratch[dev].mu, std::defer_lock);
    if (!locked) lk.lock();
    if (g_basis[dev].chunks.empty() && !g_basis[dev].logs) return false;
    if (basis_pool_release(dev) != CIQ_OK) return false;
    if (hipMalloc(p, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    *p = nullptr;
    return false;
}

// Chunk size: 2 GiB ($CIQ_BASIS_CHUNK_MIB overrides it), at least one slot.
size_t basis_chunk_bytes(size_t stride) {
    size_t mib = 2048;
    if (const char* e = std::getenv("CIQ_BASIS_CHUNK_MIB")) {
        const long v = std::strtol(e, nullptr, 10);
        if (v > 0) mib = (size_t)v;
    }
    const size_t c = std::max(mib << 20, stride);
    return (c + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);
}

// One run's slots: slot k is chunk k / per_chunk at byte offset
// (k % per_chunk) * stride. `tab` (device, max_slots entries) holds the
// pointers of the first `cap` slots; ensure() extends it on the stream (a
// small kernel writes the new entries), taking pooled chunks first and
// allocating new ones past them. Called before the launches that can reach
// a slot.
struct BasisSlots {
    int dev = 0;
    size_t stride = 0;
    int per_chunk = 0;
    int max_slots = 0;
    int cap = 0;
    double** tab = nullptr;

    double* slot(int t) const {
        return reinterpret_cast<double*>(static_cast<char*>(g_basis[dev].chunks[(size_t)t / per_chunk]) +
                                         (size_t)(t % per_chunk) * stride);
    }

    int ensure(int slots, hipStream_t st) {
        slots = std::min(slots, max_slots);
        if (slots <= cap) return CIQ_OK;
        BasisPool& bp = g_basis[dev];
        const size_t kend = basis_chunks_for(slots, per_chunk);   // chunks that cover the slots
        while (bp.chunks.size() < kend) {
            void* p = nullptr;
            if (hipMalloc(&p, bp.chunk_bytes) != hipSuccess) {
                (void)hipGetLastError();
                return CIQ_ENOMEM;
            }
            bp.chunks.push_back(p);
        }
        hipError_t e = hipSuccess;
        cap = basis_table_ranges(cap, slots, per_chunk, max_slots, kBasisChunksPerLaunch, [&](int lo, int hi, int k0) {
            if (e != hipSuccess) return;
            BasisChunks c{};
            for (int u = 0; u < kBasisChunksPerLaunch && (size_t)(k0 + u) < bp.chunks.size(); ++u)
                c.base[u] = static_cast<char*>(bp.chunks[(size_t)k0 + u]);
            e = launch_basis_table(tab, lo, hi, per_chunk, stride, k0, c, st);
        });
        HIPCHK(e);
        return CIQ_OK;
    }
};

int scratch_reserve(int dev, size_t bytes, void** out) {
    DeviceScratch& sc = g_scratch[dev];
    if (sc.cap < bytes) {
        if (sc.ptr) {
            HIPCHK(hipDeviceSynchronize());
            HIPCHK(hipFree(sc.ptr));
            sc.ptr = nullptr;
            sc.cap = 0;
        }
        size_t want = bytes + bytes / 4 + (1 << 20);
        if (hipMalloc(&sc.ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            sc.ptr = nullptr;
            if (!dev_malloc(&sc.ptr, bytes)) {
                (void)hipGetLastError();
                sc.ptr = nullptr;
                return CIQ_ENOMEM;
            }
            want = bytes;
        }
        sc.cap = want;
    }
    if (!sc.pinned) {
        if (hipHostMalloc((void**)&sc.pinned, sizeof(IterState), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            sc.pinned = nullptr;
            return CIQ_ENOMEM;
        }
    }
    *out = sc.ptr;
    return CIQ_OK;
}

// Bump allocator over the scratch area (256-byte aligned pieces).
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
};
// Same layout arithmetic without a base pointer (to size the scratch first).
struct Sizer {
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        off += count * sizeof(T);
        return nullptr;
    }
};

// Point padding: the products are instantiated for 4/6/8/10/12/16 dims, the
// gradient pass (dtype < 0) for 4/8/12/16.
int pad_dims(int d, int dtype) {
    if (dtype == CIQ_F64 || dtype == CIQ_F32)
        return d <= 4 ? 4 : d <= 6 ? 6 : d <= 8 ? 8 : d <= 10 ? 10 : d <= 12 ? 12 : 16;
    return d <= 4 ? 4 : d <= 8 ? 8 : d <= 12 ? 12 : 16;
}

// ---- kernel-product autotuner ---------------------------------------------
// Candidates: RT (16-row tiles per wave, 1 or 2; register use vs operand
// reuse) with the split of the j range that fills the chip for that RT; for
// batched runs also the number of column ranges per work item (1, 2, 4).
// Each candidate's product is timed with HIP events on the problem itself the
// first time a (device, dtype, kernel, dims, column blocks, log2 rows,
// resident, problems, accumulation) key is met. Winners are kept for the
// process and in a text file, one "key = rt nsplit" line each (lines that
// do not parse are skipped): $CIQ_TUNE_CACHE if set (empty: no file), else
// $HOME/.cache/libciq/tune.txt.
struct TuneKey {
    std::string arch;
    int dtype, kernel, dp, nsb, nlog, cached, batched, acc;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, dtype, kernel, dp, nsb, nlog, cached, batched, acc) <
               std::tie(o.arch, o.dtype, o.kernel, o.dp, o.nsb, o.nlog, o.cached, o.batched, o.acc);
    }
    std::string text() const {
        char b[256];
        std::snprintf(b, sizeof(b), "%s %d %d %d %d %d %d %d %d", arch.c_str(), dtype, kernel, dp, nsb, nlog, cached,
                      batched, acc);
        return b;
    }
};
struct TuneVal {
    int rt, nsplit;   // nsplit 0: the split rule of Run::configure
};
std::map<TuneKey, TuneVal> g_tuned;   // guarded by the device scratch lock
bool g_tune_loaded = false;

std::string tune_cache_path() {
    const char* e = std::getenv("CIQ_TUNE_CACHE");
    if (e) return std::string(e);
    const char* h = std::getenv("HOME");
    return h ? std::string(h) + "/.cache/libciq/tune.txt" : std::string();
}

void tune_cache_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    std::FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[512], arch[128];
    TuneKey k;
    TuneVal v;
    while (std::fgets(line, sizeof(line), f)) {
        if (std::sscanf(line, "%127s %d %d %d %d %d %d %d %d = %d %d", arch, &k.dtype, &k.kernel, &k.dp, &k.nsb,
                        &k.nlog, &k.cached, &k.batched, &k.acc, &v.rt, &v.nsplit) != 11)
            continue;
        k.arch = arch;
        if (v.rt >= 1 && v.rt <= 2 && v.nsplit >= 0 && v.nsplit <= 8) g_tuned[k] = v;
    }
    std::fclose(f);
}

void tune_cache_store(const TuneKey& k, const TuneVal& v) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {   // create the directory chain (best effort)
        for (size_t i = 1; i <= slash; ++i)
            if (path[i] == '/' || i == slash) (void)::mkdir(path.substr(0, i == slash ? slash : i).c_str(), 0755);
    }
    std::FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s = %d %d\n", k.text().c_str(), v.rt, v.nsplit);
    std::fclose(f);
}

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    char b[160];
    std::snprintf(b, sizeof(b), "%s/%dcu", prop.gcnArchName, prop.multiProcessorCount);
    for (char* c = b; *c; ++c)
        if (*c == ' ' || *c == '=') *c = '_';
    return b;
}

bool valid_problem(const ciq_problem* p) {
    if (!p || !p->x || !p->lengthscale) return false;
    if (p->n < 1 || p->d < 1 || p->d > CIQ_MAX_D) return false;
    if (p->kernel != CIQ_KERNEL_RBF && p->kernel != CIQ_KERNEL_MATERN52) return false;
    if (p->n_lengthscale != 1 && p->n_lengthscale != p->d) return false;
    for (int k = 0; k < p->n_lengthscale; ++k)
        if (!(p->lengthscale[k] > 0.0) || !std::isfinite(p->lengthscale[k])) return false;
    if (!(p->outputscale > 0.0) || !std::isfinite(p->outputscale)) return false;
    if (!(p->noise >= 0.0) || !std::isfinite(p->noise)) return false;
    return true;
}

bool valid_dtype(int dt) { return dt == CIQ_F64 || dt == CIQ_F32 || dt == CIQ_BF16X3 || dt == CIQ_F16X3; }

// Per-dimension multipliers applied to X so the device kernels evaluate k from
// a plain squared distance (see kfun32 / kfun64 in kernels.hip).
void point_scale(const ciq_problem* p, int dtype, double* scale) {
    (void)dtype;
    // RBF: k = exp(-r2/2) with r2 of (x/l); Matern-5/2: rho = sqrt(r2) with r2 of (sqrt5 x/l)
    const double c = (p->kernel == CIQ_KERNEL_RBF) ? 1.0 : kSqrt5;
    for (int k = 0; k < p->d; ++k) {
        const double l = p->lengthscale[p->n_lengthscale == 1 ? 0 : k];
        scale[k] = c / l;
    }
}

int get_device(int* dev) {
    HIPCHK(hipGetDevice(dev));
    if (*dev < 0 || *dev >= kMaxDevices) return CIQ_EINVAL;
    return CIQ_OK;
}

// ---- pivoted-Cholesky preconditioner (Sec. 3.4, Appendix D) -----------------
// P = Lbar Lbar^T + sigma^2 I; with Lbar^T Lbar = V diag(lam) V^T and
// U = Lbar V, P^{-1} x and P^{1/2} x are alpha0 x + U diag(f) U^T x (see
// precond.hip). Built once per call in a device allocation of its own.
constexpr double kPcholStopRtol = 1e-10;   // numerical-rank stop of the factorisation

struct DevAlloc {
    void* p = nullptr;
    ~DevAlloc() {
        if (p) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
        }
    }
};

// Bump allocation inside one device buffer (256-byte aligned pieces).
template <typename T>
T* carve(char* base, size_t& off, size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
}

struct Precond {
    int R = 0;              // columns of U (requested rank, at most n)
    int rank = 0;           // pivots the factorisation took
    double s2 = 0.0;        // sigma^2
    double trace = 0.0;     // trace of Ktil - Lbar Lbar^T
    double* U = nullptr;    // n x R
    double* fin = nullptr;  // [R] weights of P^{-1}
    double* fsq = nullptr;  // [R] weights of P^{1/2}
    double* part = nullptr; // low-rank partials
    double* T = nullptr;    // R x max(s, R)
    double* dotp = nullptr; // [apply blocks][s]
    DevAlloc mem;
};

int pchol_blocks(int n) { return std::max(1, std::min((n + 255) / 256, 2048)); }

// Scratch of one factorisation (L itself is the caller's).
struct PcholScratch {
    double *dres, *pval, *trace, *bval, *bsum;
    int *chosen, *piv, *bidx;
};
template <typename F>
void pchol_layout(int n, int R, F&& take_d, PcholScratch& w) {
    const int nblk = pchol_blocks(n);
    w.dres = take_d((size_t)n);
    w.pval = take_d((size_t)R + 1);
    w.trace = take_d((size_t)R + 1);
    w.bval = take_d((size_t)nblk);
    w.bsum = take_d((size_t)nblk);
    // integer arrays as doubles' worth of space (8 bytes per entry)
    w.chosen = reinterpret_cast<int*>(take_d((size_t)n));
    w.piv = reinterpret_cast<int*>(take_d((size_t)R + 1));
    w.bidx = reinterpret_cast<int*>(take_d((size_t)nblk));
}

// Rank-R factor into L (n x ldl, zero-filled here); pivots and the final
// residual trace to the host. Synchronous.
int pchol_run(const double* xh, int n, int dp, int kernel, int ard, const double* scale, double o2, int R,
              double* L, int ldl, const PcholScratch& w, std::vector<int>& piv, double* trace, hipStream_t st) {
    PcholArgs a{};
    a.xh = xh;
    for (int k = 0; k < CIQ_MAX_D; ++k) a.scale[k] = scale[k];
    a.n = n;
    a.dp = dp;
    a.kernel = kernel;
    a.ard = ard;
    a.o2 = o2;
    a.stop_abs = kPcholStopRtol * o2;
    a.L = L;
    a.ldl = ldl;
    a.dres = w.dres;
    a.chosen = w.chosen;
    a.piv = w.piv;
    a.pval = w.pval;
    a.trace = w.trace;
    a.bval = w.bval;
    a.bidx = w.bidx;
    a.bsum = w.bsum;
    a.nblk = pchol_blocks(n);
    HIPCHK(launch_fill<double>(L, (size_t)n * ldl, 0.0, st));
    HIPCHK(launch_pchol_init(a, st));
    for (int m = 0; m < R; ++m) {
        HIPCHK(launch_pchol_pick(a, m, st));
        HIPCHK(launch_pchol_col(a, m, st));
    }
    HIPCHK(launch_pchol_pick(a, R, st));
    piv.assign((size_t)R, -1);
    HIPCHK(hipMemcpyAsync(piv.data(), w.piv, (size_t)R * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(trace, w.trace + R, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return CIQ_OK;
}

// Y = alpha0 X + U diag(f) U^T X for X, Y n x S (ld S; Y may be X).
int pc_apply(const Precond& pc, double alpha0, const double* f, const double* X, int n, int S, double* Y,
             double* dotp, const int* colmask, const int* done, hipStream_t st) {
    const int nch = lr_part_chunks(n, pc.R, S);
    HIPCHK(launch_lr_part(pc.U, pc.R, X, S, n, pc.R, S, nch, pc.part, done, st));
    HIPCHK(launch_lr_reduce(pc.part, nch, pc.R, S, f, pc.T, S, done, st));
    HIPCHK(launch_lr_apply(alpha0, X, S, pc.U, pc.R, pc.T, S, n, pc.R, S, Y, S, dotp, colmask, done, st));
    return CIQ_OK;
}

// Factorisation, Gram matrix, its eigendecomposition (host, Householder +
// implicit QR) and U = Lbar V for one problem whose FP64 points are xh (n x dp).
int pc_build(const ciq_problem& p, const double* xh, int dp, int kernel, int ard, const double* scale, int rank,
             int s_cap, Precond& pc, hipStream_t st) {
    const int n = p.n;
    const int R = std::min(rank, n);
    pc.R = R;
    pc.s2 = p.noise;
    // partial buffer for the widths it serves: s_cap (solve), 1 (bounds), R (Gram)
    size_t part_n = 0;
    for (int w : {s_cap, 1, R}) part_n = std::max(part_n, (size_t)lr_part_chunks(n, R, w) * R * w);
    size_t off = 0;
    PcholScratch w{};
    auto layout = [&](char* base) {
        off = 0;
        pc.U = carve<double>(base, off, (size_t)n * R);
        double* L = carve<double>(base, off, (size_t)n * R);
        pc.fin = carve<double>(base, off, R);
        pc.fsq = carve<double>(base, off, R);
        pc.part = carve<double>(base, off, part_n);
        pc.T = carve<double>(base, off, (size_t)R * std::max(s_cap, R));
        pc.dotp = carve<double>(base, off, (size_t)lr_apply_blocks(n) * s_cap);
        pchol_layout(n, R, [&](size_t c) { return carve<double>(base, off, c); }, w);
        return L;
    };
    layout(nullptr);
    if (!dev_malloc(&pc.mem.p, off)) {
        (void)hipGetLastError();
        pc.mem.p = nullptr;
        return CIQ_ENOMEM;
    }
    double* L = layout(static_cast<char*>(pc.mem.p));
    std::vector<int> piv;
    STCHK(pchol_run(xh, n, dp, kernel, ard, scale, p.outputscale, R, L, R, w, piv, &pc.trace, st));
    pc.rank = 0;
    for (int v : piv) pc.rank += (v >= 0) ? 1 : 0;
    // Gram matrix Lbar^T Lbar (R x R) and its eigendecomposition
    const int nch = lr_part_chunks(n, R, R);
    HIPCHK(launch_lr_part(L, R, L, R, n, R, R, nch, pc.part, nullptr, st));
    HIPCHK(launch_lr_reduce(pc.part, nch, R, R, nullptr, pc.T, R, nullptr, st));
    std::vector<double> G((size_t)R * R), lam, V;
    HIPCHK(hipMemcpyAsync(G.data(), pc.T, G.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < R; ++i)
        for (int j = i + 1; j < R; ++j) {
            const double m = 0.5 * (G[(size_t)i * R + j] + G[(size_t)j * R + i]);
            G[(size_t)i * R + j] = G[(size_t)j * R + i] = m;
        }
    sym_eig_tridiag(R, G, lam, V);
    std::vector<double> fin(R), fsq(R);
    const double s2 = p.noise, sg = std::sqrt(p.noise);
    for (int r = 0; r < R; ++r) {
        const double l = std::max(lam[r], 0.0);
        fin[r] = -1.0 / (s2 * (l + s2));
        fsq[r] = 1.0 / (std::sqrt(l + s2) + sg);
    }
    HIPCHK(hipMemcpyAsync(pc.T, V.data(), V.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(pc.fin, fin.data(), R * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(pc.fsq, fsq.data(), R * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(launch_lr_apply(0.0, nullptr, 0, L, R, pc.T, R, n, R, R, pc.U, R, nullptr, nullptr, nullptr, st));
    HIPCHK(hipStreamSynchronize(st));   // host vectors are pageable and short-lived
    return CIQ_OK;
}

// ---- posterior covariance at a candidate set (Sec. 5.2) ---------------------
// Sigma = Kss + jitter I - W W^T with W = Ksx L^{-T}, L L^T = Kxx + sigma_obs^2 I
// (blocked Cholesky of the observation block and the triangular solve for W
// on the device, chol.hip). Every product with
// Sigma is the candidate kernel product plus the low-rank correction
// -W (W^T v), accumulated into the product's first partial.
struct PostSpec {
    const void* x_obs;   // device, n_obs x d (element type of the candidates' X)
    int n_obs;
    double obs_noise;
};

struct Posterior {
    int n = 0;              // observations
    int ldw = 0;            // leading dimension of W: n rounded up to 64
    double* W = nullptr;    // T x ldw (columns n.. zero)
    double* fneg = nullptr; // [n] of -1
    double* part = nullptr; // low-rank partials
    double* T = nullptr;    // n x s
    DevAlloc mem;
};

// Sigma's correction for candidates with FP64 points xh (T x dp): Kxx and
// Ksx into blocks padded to npad = 64 ceil(n / 64) columns, the factor and
// W = Ksx L^{-T} (in place of Ksx) on the device. Synchronous.
int post_build(const ciq_problem& cand, int dtype, const double* xh, int dp, int kernel, int ard,
               const double* scale, const PostSpec& ps, int s_cap, Posterior& po, hipStream_t st) {
    const int T = cand.n, n = ps.n_obs;
    const int npad = (n + 63) / 64 * 64;
    po.n = n;
    po.ldw = npad;
    size_t part_n = 0;
    for (int w : {s_cap, 1}) part_n = std::max(part_n, (size_t)lr_part_chunks(T, n, w) * n * w);
    size_t off = 0;
    double *xo = nullptr, *kxx = nullptr, *dinv = nullptr;
    int* status = nullptr;
    auto layout = [&](char* base) {
        off = 0;
        po.W = carve<double>(base, off, (size_t)T * npad);
        xo = carve<double>(base, off, (size_t)n * dp);
        kxx = carve<double>(base, off, (size_t)npad * npad);
        dinv = carve<double>(base, off, (size_t)npad * 64);
        status = reinterpret_cast<int*>(carve<double>(base, off, 1));
        po.fneg = carve<double>(base, off, n);
        po.part = carve<double>(base, off, part_n);
        po.T = carve<double>(base, off, (size_t)n * s_cap);
    };
    layout(nullptr);
    if (!dev_malloc(&po.mem.p, off)) {
        (void)hipGetLastError();
        po.mem.p = nullptr;
        return CIQ_ENOMEM;
    }
    layout(static_cast<char*>(po.mem.p));
    double ones[CIQ_MAX_D];
    for (int k = 0; k < CIQ_MAX_D; ++k) ones[k] = 1.0;
    if (dtype == CIQ_F64)
        HIPCHK(launch_prep<double>(static_cast<const double*>(ps.x_obs), n, cand.d, dp, ones, xo, st));
    else
        HIPCHK(launch_prep<float>(static_cast<const float*>(ps.x_obs), n, cand.d, dp, ones, xo, st));
    HIPCHK(launch_fill<double>(kxx, (size_t)npad * npad, 0.0, st));
    HIPCHK(launch_xkernel(xo, n, xo, n, dp, kernel, ard, scale, cand.outputscale, kxx, npad, st));
    HIPCHK(launch_chol_prep(kxx, n, npad, ps.obs_noise, st));
    if (npad > n) HIPCHK(launch_fill<double>(po.W, (size_t)T * npad, 0.0, st));
    HIPCHK(launch_xkernel(xh, T, xo, n, dp, kernel, ard, scale, cand.outputscale, po.W, npad, st));
    HIPCHK(launch_fill<double>(po.fneg, n, -1.0, st));
    HIPCHK(launch_fill<int>(status, 1, 0, st));
    HIPCHK(launch_chol_blocked(kxx, npad, dinv, status, st));
    HIPCHK(launch_trsm_right_lt(po.W, T, npad, kxx, dinv, st));
    int h_status = 0;
    HIPCHK(hipMemcpyAsync(&h_status, status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return h_status ? CIQ_ENUMERIC : CIQ_OK;
}

// ---------------------------------------------------------------------------
// One Krylov run over nprob problems (the single-problem calls use nprob = 1).
// ---------------------------------------------------------------------------
template <typename T>
struct Run {
    int dtype = CIQ_F32, kernel = 0, dp = 4;
    int nprob = 1, s = 1, Q = 0, max_iter = 0, rows_total = 0, max_n = 0;
    double tol = 0.0;
    int bounds_mode = 0;
    int nsplit = 1, nrb = 0, rt = 2, nsplit_alloc = 1, nrb_alloc = 1;
    int nsplit_fixed = 0;    // batched: column ranges per work item chosen by the tuner (0: the rule below)
    int* queue = nullptr;    // batched FP32: persistent product's work counter
    long long* pkt = nullptr;    // batched resident FP32: per-problem matrix offsets (elements)
    long long* pnjs = nullptr;   // per-problem padded columns / 4
    bool keep_solves = false;
    int fine_acc = 0;      // FP32 resident products: the finer FP64 accumulation (inverse root)
    bool cached = false;   // products stream a resident kernel matrix (kt)
    bool precond = false;  // preconditioned run (single problem): Lanczos in the P^{-1} inner product
    const Precond* pc = nullptr;
    BasisSlots* bslots = nullptr;   // resident Krylov basis of this run (d.basis is its table)
    const Posterior* post = nullptr;   // products with a posterior covariance (single problem)
    const SparseOp* sp = nullptr;      // products with a caller's sparse operator (single problem, FP64)
    const DenseOp* dn = nullptr;       // products with a dense operator (single-shift solves, FP64)
    // device memory: points in FP64, every msMINRES vector in FP64
    // (FP32 Lanczos vectors cost ~eps32 * kappa accuracy; the FP32 product only
    // consumes an FP32 copy q32 of the current Lanczos vector)
    double* xh = nullptr;
    double* qbuf[2] = {nullptr, nullptr};
    double* ypart = nullptr;
    double* mbuf[2] = {nullptr, nullptr};
    double* acc = nullptr;
    double* solves = nullptr;  // [rows][Q][s]
    float* q32 = nullptr;      // FP32 product operand (T = float only)
    double* pbuf[2] = {nullptr, nullptr};  // preconditioned: p_j = P^{-1} z_j (qbuf holds z_j)
    WorkItem* wl = nullptr;
    int* pn = nullptr;
    int* poff = nullptr;
    float* po2 = nullptr;
    float* ps2 = nullptr;
    double* pscale = nullptr;  // [nprob][CIQ_MAX_D] FP32-product difference scales
    double* t = nullptr;
    double* w = nullptr;
    const void* kt = nullptr;    // resident kernel matrix (single problem) or nullptr
    long long njs = 0;
    // split FP16 resident products (CIQ_F16X3): tiled operand copy of q_j / p_j
    void* vt16 = nullptr;
    int nsbt = 0;
    float op_scale = kOp16Scale;
    double* opsc = nullptr;      // [s] per-column scales of an arbitrary operand (final product)
    double* opinv = nullptr;
    Dev d{};
    long long ysplit = 0;
    // square root's main loop on a resident FP32 / split-FP16 matrix (one
    // problem, no preconditioner, posterior or caller operator): the product
    // writes FP32 split partials, which phase 0 sums in FP64 (see solve)
    bool part32 = false;
    float* ypart32 = nullptr;
    // host mirrors
    std::vector<int> h_n, h_off;
    std::vector<float> h_o2, h_s2;
    std::vector<double> h_scale;
    std::vector<double> h_o2d, h_s2d;
    std::vector<long long> h_pkt, h_pnjs;
    int ard = 0;

    template <typename A>
    void layout(A& a, bool with_xh) {
        const int ncol = nprob * s;
        const size_t vec = (size_t)rows_total * s;
        if (with_xh) xh = a.template take<double>((size_t)rows_total * dp);
        qbuf[0] = a.template take<double>(vec);
        qbuf[1] = a.template take<double>(vec);
        ypart = a.template take<double>(vec * nsplit_alloc);
        if (part32) ypart32 = a.template take<float>(vec * nsplit_alloc);
        if (Q > 0) {
            mbuf[0] = a.template take<double>(vec * Q);
            mbuf[1] = a.template take<double>(vec * Q);
        }
        acc = a.template take<double>(vec);
        if (keep_solves) solves = a.template take<double>(vec * Q);
        if (f16_resident()) {
            nsbt = op16_nsbt(s);
            vt16 = a.template take<_Float16>(op16_halfs(kcache_cols(max_n), nsbt));
            opsc = a.template take<double>(s);
            opinv = a.template take<double>(s);
        } else if (sizeof(T) == 4) {
            q32 = a.template take<float>(vec);
        }
        if (precond) {
            pbuf[0] = a.template take<double>(vec);
            pbuf[1] = a.template take<double>(vec);
        }
        wl = a.template take<WorkItem>(std::max(nrb_alloc, 1));
        queue = a.template take<int>(1);
        pkt = a.template take<long long>(nprob);
        pnjs = a.template take<long long>(nprob);
        pn = a.template take<int>(nprob);
        poff = a.template take<int>(nprob);
        po2 = a.template take<float>(nprob);
        ps2 = a.template take<float>(nprob);
        pscale = a.template take<double>((size_t)nprob * CIQ_MAX_D);
        t = a.template take<double>(std::max(nprob * Q, 1));
        w = a.template take<double>(std::max(nprob * Q, 1));
        d.dots = a.template take<double>((size_t)nprob * d.dots_blocks * s * 2);
        d.colsum = a.template take<double>((size_t)2 * ncol);
        d.beta1 = a.template take<double>(ncol);
        d.beta_cur = a.template take<double>(ncol);
        d.alpha = a.template take<double>(ncol);
        d.beta_next = a.template take<double>(ncol);
        d.inv_beta_next = a.template take<double>(ncol);
        d.beta_used = a.template take<double>(ncol);
        d.colflag = a.template take<int>(ncol);
        d.colactive = a.template take<int>(ncol);
        d.col_iters = a.template take<int>(ncol);
        d.prob_done = a.template take<int>(nprob);
        d.T = bounds_mode ? a.template take<double>((size_t)std::max(max_iter, 1) * ncol * 2) : nullptr;
        const size_t qn = (size_t)std::max(Q, 1) * ncol;
        d.c1 = a.template take<double>(qn);
        d.s1 = a.template take<double>(qn);
        d.c2 = a.template take<double>(qn);
        d.s2 = a.template take<double>(qn);
        d.phibar = a.template take<double>(qn);
        d.relres = a.template take<double>(qn);
        d.frozen = a.template take<int>(qn);
        d.coef = a.template take<ShiftCoef>(qn);
        d.st = a.template take<IterState>(1);
    }

    int rows_per_block() const { return cached ? 64 * rt : mvm_rows_per_block(dtype, s, rt); }
    bool f16_resident() const { return dtype == CIQ_F16X3 && cached; }

    void configure(int rt_) {
        rt = rt_;
        {   // ~8 rows per thread in the inner-product kernels, at most 512
            // blocks: their partials are summed per column by single-block
            // stages, and at N = 50,000, S = 64 a step with 512 blocks takes
            // 12-14 us less than with 1024 (256 leave the passes short of
            // loads in flight; measured). The scalar stage sums both inner
            // products' block partials itself; with few blocks phase 1 sums
            // the alpha partials itself too. The preconditioned step reads
            // the block-summed alpha (colsum) and writes beta^2 there itself.
            int ts = 1;
            while (ts < s && ts < 64) ts <<= 1;
            const int rows_per_pass = 256 / ts;
            d.dots_blocks = std::min(512, std::max(1, (max_n + rows_per_pass * 8 - 1) / (rows_per_pass * 8)));
            d.fuse_sums = precond ? 0 : (d.dots_blocks <= 32 ? 3 : 1);
        }
        const int rpb = rows_per_block();
        nrb = 0;
        for (int p = 0; p < nprob; ++p) nrb += (h_n[p] + rpb - 1) / rpb;
        nsplit = mvm_pick_nsplit(dtype, nrb, max_n, s);
        if (cached && (max_n + 63) / 64 >= 16 && nrb * 8 >= 512) {
            // m column ranges per XCD (split = block index mod 8 picks the XCD):
            // m = 2 when it fills the last round of equal-cost blocks on the
            // XCD's 32 CUs enough to pay for 8 more partial products (each
            // one more N x S FP64 write and read, ~0.2 % of a product); at
            // most 2, so the V slices an XCD streams stay within its L2
            const int nsb = (std::min(s, product_cap(dtype, true)) + 15) / 16;
            const int bpc = kt_blocks_per_cu(dtype, nsb, rt, fine_acc);
            int m = 1;
            if (bpc > 0) {
                const double slots = 32.0 * bpc;
                auto fill = [&](int mm) {
                    const double work = (double)nrb * mm;
                    return work / (std::ceil(work / slots) * slots) - 0.002 * 8 * (mm - 1);
                };
                if (fill(2) > fill(1) + 0.01) m = 2;
            }
            nsplit = 8 * m;
        } else if (cached && (max_n + 63) / 64 >= 8 && nrb * 8 >= 512) {
            nsplit = 8;   // one column range per XCD
        }
        if (nprob > 1 && nsplit_fixed > 0) nsplit = nsplit_fixed;
        if (sp || dn) nsplit = 1;   // the sparse / dense products write one partial
        ysplit = (long long)rows_total * s;
    }

    // size the partial-product buffer and the work list for every RT candidate
    void plan(int rt_) {
        nsplit_alloc = 1;
        nrb_alloc = 1;
        for (int r = 1; r <= 2; ++r) {
            configure(r);
            nsplit_alloc = std::max(nsplit_alloc, nsplit);
            nrb_alloc = std::max(nrb_alloc, nrb);
        }
        if (nprob > 1) nsplit_alloc = std::max(nsplit_alloc, 4);   // the tuner's batched candidates
        configure(rt_);
    }

    void fill_dev() {
        d.nprob = nprob;
        d.s = s;
        d.Q = Q;
        d.ncol = nprob * s;
        d.max_iter = max_iter;
        d.rows_total = rows_total;
        d.n = pn;
        d.row_off = poff;
        d.t = t;
        d.w = w;
        d.tol = tol;
        d.bd_rtol = (dtype == CIQ_F64) ? 1e-13 : 1e-6;
        d.bounds_mode = bounds_mode;
    }

    // Work list: every problem's row blocks, largest problem first (its items
    // cost the most; the persistent product takes them in list order, so the
    // small items fill the end of the launch).
    int upload_tables(hipStream_t st) {
        const int rpb = rows_per_block();
        std::vector<int> order(nprob);
        for (int p = 0; p < nprob; ++p) order[p] = p;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return h_n[x] > h_n[y]; });
        std::vector<WorkItem> h_wl;
        for (int p : order) {
            const int nb = (h_n[p] + rpb - 1) / rpb;
            for (int r = 0; r < nb; ++r) h_wl.push_back(WorkItem{p, r});
        }
        HIPCHK(hipMemcpyAsync(wl, h_wl.data(), h_wl.size() * sizeof(WorkItem), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(pn, h_n.data(), nprob * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(poff, h_off.data(), nprob * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(po2, h_o2.data(), nprob * sizeof(float), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(ps2, h_s2.data(), nprob * sizeof(float), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(pscale, h_scale.data(), h_scale.size() * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(pkt, h_pkt.data(), nprob * sizeof(long long), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(pnjs, h_pnjs.data(), nprob * sizeof(long long), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));  // host vectors are pageable and short-lived
        return CIQ_OK;
    }

    MvmArgs mvm_args(const void* v, double* y) const {
        MvmArgs a{};
        a.xh = xh;
        a.v = v;
        a.y = y;
        a.ysplit = ysplit;
        a.ldv = s;
        a.ldy = s;
        a.s = s;
        a.kernel = kernel;
        a.dp = dp;
        a.nsplit = nsplit;
        a.rt = rt;
        a.acc = fine_acc;
        a.ard = ard;
        for (int k = 0; k < CIQ_MAX_D; ++k) a.scale[k] = h_scale[k];
        a.pscale = pscale;
        a.n = h_n[0];
        a.o2 = h_o2d[0];
        a.s2 = h_s2d[0];
        a.wl = (nprob > 1) ? wl : nullptr;
        a.nrb = nrb;
        a.pn = pn;
        a.poff = poff;
        a.po2 = po2;
        a.ps2 = ps2;
        a.prob_done = (nprob > 1) ? d.prob_done : nullptr;
        a.done = &d.st->done;
        a.queue = (nprob > 1 && dtype == CIQ_F32) ? queue : nullptr;
        a.nitems = nrb * nsplit;
        a.pkt = (nprob > 1) ? pkt : nullptr;
        a.pnjs = (nprob > 1) ? pnjs : nullptr;
        a.kt = kt;
        a.njs = njs;
        a.vt = vt16;
        a.nsbt = nsbt;
        a.vinv = 1.0 / (double)op_scale;
        a.vcol_inv = nullptr;
        return a;
    }

    // Operand of iteration j's kernel product: q_j (p_j when preconditioned),
    // or its FP32 copy.
    const void* operand(int j) const {
        if (q32) return q32;
        return precond ? pbuf[(j - 1) & 1] : qbuf[(j - 1) & 1];   // (split FP16: the noise term's)
    }
    Op16 op16() const { return Op16{vt16, nsbt, op_scale}; }

    // Iteration j's kernels after the product (the buffer roles depend on the
    // parity of j only).
    int enqueue_post(int j, hipStream_t st) {
        double* qcur = qbuf[(j - 1) & 1];
        double* qprv = qbuf[j & 1];
        double* mcur = mbuf[j & 1];       // holds m_{j-2}, receives m_j
        double* mprv = mbuf[(j - 1) & 1];  // holds m_{j-1}
        if (precond) {
            // Appendix D: alpha_j = p_j^T (K p_j - beta_j z_{j-1}),
            // w = K p_j - beta_j z_{j-1} - alpha_j z_j, P^{-1} w, beta_{j+1}^2 = w^T P^{-1} w
            double* pcur = pbuf[(j - 1) & 1];
            double* pnxt = pbuf[j & 1];
            const int* done = &d.st->done;
            HIPCHK(launch_dots<double>(d, ypart, ysplit, nsplit, pcur, qprv, 0, st));   // also reduces
            HIPCHK(launch_colsum(d, 0, st));
            HIPCHK(launch_pc_w(d, ypart, qcur, qprv, st));
            STCHK(pc_apply(*pc, 1.0 / pc->s2, pc->fin, ypart, rows_total, s, pnxt, pc->dotp, d.colactive, done,
                           st));
            HIPCHK(launch_lr_dotsum(pc->dotp, lr_apply_blocks(rows_total), s, d.colsum + d.ncol, done, st));
            HIPCHK(launch_scalar(d, st));
            HIPCHK(launch_update<double>(d, ypart, ysplit, 1, pcur, qprv, mprv, mcur, acc, solves, q32, max_n, st,
                                         pnxt, op16()));
            return CIQ_OK;
        }
        HIPCHK(launch_dots<double>(d, ypart, ysplit, nsplit, qcur, qprv, 0, st,   // also reduces the splits
                                   (part32 && nsplit > 1) ? ypart32 : nullptr));
        HIPCHK(launch_colsum(d, 0, st));
        HIPCHK(launch_dots<double>(d, ypart, ysplit, 1, qcur, qprv, 1, st));
        HIPCHK(launch_colsum(d, 1, st));
        HIPCHK(launch_scalar(d, st));
        HIPCHK(launch_update<double>(d, ypart, ysplit, 1, qcur, qprv, mprv, mcur, acc, solves, q32, max_n, st,
                                     nullptr, op16()));
        return CIQ_OK;
    }

    // Posterior covariance: the product's first partial += -W (W^T v) for the
    // FP64 operand v (rows_total x s).
    int post_correct(const double* v, const int* done, hipStream_t st) {
        if (!post) return CIQ_OK;
        const int nch = lr_part_chunks(rows_total, post->n, s);
        HIPCHK(launch_lr_part(post->W, post->ldw, v, s, rows_total, post->n, s, nch, post->part, done, st));
        HIPCHK(launch_lr_reduce(post->part, nch, post->n, s, post->fneg, post->T, s, done, st));
        HIPCHK(launch_lr_apply(0.0, nullptr, 0, post->W, post->ldw, post->T, s, rows_total, post->n, s, ypart, s,
                               nullptr, nullptr, done, st, 1));
        return CIQ_OK;
    }

    // The product of iteration j (kernel matrix, or the caller's sparse operator).
    int product(int j, hipStream_t st) {
        if (sp) {
            HIPCHK(launch_spmv(*sp, qbuf[(j - 1) & 1], s, s, ypart, s, &d.st->done, st));
            return CIQ_OK;
        }
        if (dn) {
            HIPCHK(launch_lr_apply(0.0, nullptr, 0, dn->A, dn->n, qbuf[(j - 1) & 1], s, rows_total, dn->n, s, ypart,
                                   s, nullptr, nullptr, &d.st->done, st));
            return CIQ_OK;
        }
        MvmArgs a = mvm_args(operand(j), ypart);
        if (part32 && nsplit > 1) a.y32 = ypart32;
        HIPCHK(launch_mvm(dtype, a, st));
        return CIQ_OK;
    }

    // One msMINRES iteration's kernels.
    int enqueue_iteration(int j, hipStream_t st) {
        STCHK(product(j, st));
        STCHK(post_correct(qbuf[(j - 1) & 1], &d.st->done, st));
        return enqueue_post(j, st);
    }

    // Krylov iterations after the start vectors are in qbuf[0]. Returns status.
    // With use_graph, iterations (2k+1, 2k+2) are captured once into a HIP
    // graph on a private stream and the graph is launched on `st` once per two
    // iterations; kernels after the stop (or past max_iter) exit at once, so the
    // replays are the same work as the eager loop.
    int iterate(hipStream_t st, int check_every, IterState* pinned, int* mvm_count,
                hipEvent_t* ev_pool, int n_ev, double* mvm_ms, int* mvm_timed, bool use_graph = false) {
        // $CIQ_PROGRESS set: a line on stderr with the iteration count at the
        // host's convergence checks, at most one per 10 s (long solves)
        static const bool progress = std::getenv("CIQ_PROGRESS") != nullptr;
        auto last = std::chrono::steady_clock::now();
        auto report = [&]() {
            if (!progress) return;
            const auto now = std::chrono::steady_clock::now();
            if (std::chrono::duration<double>(now - last).count() < 10.0) return;
            last = now;
            std::fprintf(stderr, "[ciq] iteration %d of at most %d\n", pinned->iter, max_iter);
            std::fflush(stderr);
        };
        // the state is reused scratch: clear `done` before the first kernel that reads it
        HIPCHK(launch_fill<int>(reinterpret_cast<int*>(d.st), sizeof(IterState) / sizeof(int), 0, st));
        if (vt16)      // rows past n and columns past s of the split operand stay zero
            HIPCHK(launch_fill<int>(static_cast<int*>(vt16), op16_halfs(kcache_cols(max_n), nsbt) / 2, 0, st));
        if (precond) {
            // start z_1 = c / beta_1, p_1 = P^{-1} c / beta_1, beta_1^2 = c^T P^{-1} c
            STCHK(pc_apply(*pc, 1.0 / pc->s2, pc->fin, qbuf[0], rows_total, s, pbuf[0], pc->dotp, nullptr, nullptr,
                           st));
            HIPCHK(launch_lr_dotsum(pc->dotp, lr_apply_blocks(rows_total), s, d.colsum + d.ncol, nullptr, st));
        } else {
            HIPCHK(launch_dots<double>(d, qbuf[0], 0, 1, nullptr, nullptr, 1, st));
            HIPCHK(launch_colsum(d, 1, st));
        }
        HIPCHK(launch_scalar_init(d, st));
        if (Q > 0 && d.basis == nullptr) {   // the direction recurrence's m_{-1}, m_0
            HIPCHK(launch_fill<double>(mbuf[0], (size_t)rows_total * s * Q, 0.0, st));
            HIPCHK(launch_fill<double>(mbuf[1], (size_t)rows_total * s * Q, 0.0, st));
        }
        if (solves) HIPCHK(launch_fill<double>(solves, (size_t)rows_total * s * Q, 0.0, st));
        HIPCHK(launch_init_vectors<double>(d, qbuf[0], qbuf[1], acc, q32, rows_total, st,
                                           precond ? pbuf[0] : nullptr, op16()));
        if (bslots) {   // slot 0: q_1
            STCHK(bslots->ensure(1, st));
            HIPCHK(hipMemcpyAsync(bslots->slot(0), qbuf[0], (size_t)rows_total * s * sizeof(double),
                                  hipMemcpyDeviceToDevice, st));
        }
        if (use_graph && ev_pool == nullptr) {
            hipStream_t cs = nullptr;
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            struct Guard {
                hipStream_t& cs;
                hipGraph_t& g;
                hipGraphExec_t& e;
                ~Guard() {
                    if (e) (void)hipGraphExecDestroy(e);
                    if (g) (void)hipGraphDestroy(g);
                    if (cs) (void)hipStreamDestroy(cs);
                }
            } guard{cs, graph, exec};
            HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_iteration(1, cs);
            if (rc == CIQ_OK) rc = enqueue_iteration(2, cs);
            const hipError_t ec = hipStreamEndCapture(cs, &graph);
            if (rc != CIQ_OK) return rc;
            HIPCHK(ec);
            HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            const int per_poll = std::max(1, check_every / 2);
            int launched = 0;   // graph launches (2 iterations each)
            while (2 * launched < max_iter) {
                if (bslots) STCHK(bslots->ensure(2 * launched + 3, st));   // slots up to iteration 2 launched + 2
                HIPCHK(hipGraphLaunch(exec, st));
                ++launched;
                if (launched % per_poll == 0 || 2 * launched >= max_iter) {
                    HIPCHK(hipMemcpyAsync(pinned, d.st, sizeof(IterState), hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                    if (pinned->numeric) return CIQ_ENUMERIC;
                    if (pinned->done) break;
                    report();
                }
            }
        } else {
            int j = 1;
            int pending = 0;
            while (j <= max_iter) {
                const bool timed = ev_pool != nullptr && pending < n_ev;
                if (bslots) STCHK(bslots->ensure(j + 1, st));   // slots 0..j
                if (timed) HIPCHK(hipEventRecord(ev_pool[2 * pending], st));
                STCHK(product(j, st));
                if (timed) {
                    HIPCHK(hipEventRecord(ev_pool[2 * pending + 1], st));
                    ++pending;
                }
                STCHK(post_correct(qbuf[(j - 1) & 1], &d.st->done, st));
                STCHK(enqueue_post(j, st));
                if (j % check_every == 0 || j == max_iter) {
                    HIPCHK(hipMemcpyAsync(pinned, d.st, sizeof(IterState), hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                    if (ev_pool) {
                        // only launches issued while the run was still live count; the
                        // device-side early exit after `done` is not a kernel product
                        const int live = std::min(pending, pinned->iter - *mvm_timed);
                        for (int k = 0; k < live; ++k) {
                            float ms = 0.f;
                            HIPCHK(hipEventElapsedTime(&ms, ev_pool[2 * k], ev_pool[2 * k + 1]));
                            *mvm_ms += ms;
                        }
                        *mvm_timed += std::max(live, 0);
                        pending = 0;
                    }
                    if (pinned->numeric) return CIQ_ENUMERIC;
                    if (pinned->done) break;
                    report();
                }
                ++j;
            }
        }
        HIPCHK(hipMemcpyAsync(pinned, d.st, sizeof(IterState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (pinned->numeric) return CIQ_ENUMERIC;
        *mvm_count += pinned->iter;
        return CIQ_OK;
    }

    // Slot of the final iterate's Lanczos vector etc. is irrelevant to callers:
    // the combined solution lives in acc, the per-shift solves in `solves`.
};

// Pick RT (and for batched runs the column ranges per item) for this run
// (see TuneKey). `operand` holds any n x s data in the product's input type;
// the timed launches write only the partial buffer.
template <typename T>
int tune_rt(Run<T>& r, const void* operand, hipStream_t st) {
    if (r.sp || r.dn) {
        r.configure(1);
        return CIQ_OK;
    }
    const int nsb = (std::min(r.s, product_cap(r.dtype, r.cached)) + 15) / 16;
    const bool batched = r.nprob > 1;
    // one row tile per wave: the widest FP32 on-the-fly and split FP16 resident
    // launches (register budget) and the on-the-fly split forms
    const bool rt1 = (r.dtype == CIQ_F32 && nsb >= 8) || (r.dtype == CIQ_F16X3 && r.cached && nsb > 4) ||
                     r.dtype == CIQ_BF16X3 || (r.dtype == CIQ_F16X3 && !r.cached);
    if (rt1 && !batched) {
        r.configure(1);
        return CIQ_OK;
    }
    int nlog = 0;
    while ((1 << (nlog + 1)) <= r.rows_total) ++nlog;
    tune_cache_load();
    const TuneKey key{device_arch(), r.dtype, r.kernel, r.dp, nsb, nlog, r.cached ? 1 : 0, batched ? 1 : 0,
                      r.fine_acc};
    auto it = g_tuned.find(key);
    if (it == g_tuned.end()) {
        std::vector<TuneVal> cands;
        for (int rt = 1; rt <= (rt1 ? 1 : 2); ++rt) {
            if (batched)
                for (int ns : {1, 2, 4}) cands.push_back(TuneVal{rt, ns});
            else
                cands.push_back(TuneVal{rt, 0});
        }
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        float best_ms = 1e30f;
        TuneVal best = cands.back();
        for (const TuneVal& c : cands) {
            r.nsplit_fixed = c.nsplit;
            r.configure(c.rt);
            if (batched) STCHK(r.upload_tables(st));
            MvmArgs a = r.mvm_args(operand, r.ypart);
            a.done = nullptr;
            a.prob_done = nullptr;
            HIPCHK(launch_mvm(r.dtype, a, st));   // warm-up
            HIPCHK(hipEventRecord(e0, st));
            for (int k = 0; k < 2; ++k) HIPCHK(launch_mvm(r.dtype, a, st));
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        it = g_tuned.emplace(key, best).first;
        tune_cache_store(key, best);
    }
    r.nsplit_fixed = it->second.nsplit;
    r.configure(it->second.rt);
    return batched ? r.upload_tables(st) : CIQ_OK;
}

template <typename T>
int setup_points(Run<T>& r, const ciq_problem* probs, int dtype, hipStream_t st) {
    for (int p = 0; p < r.nprob; ++p) {
        double scale[CIQ_MAX_D];
        point_scale(&probs[p], dtype, scale);
        for (int k = 0; k < CIQ_MAX_D; ++k) scale[k] = 1.0;   // products scale differences
        HIPCHK(launch_prep<T>(static_cast<const T*>(probs[p].x), probs[p].n, probs[p].d, r.dp, scale,
                              r.xh + (size_t)r.h_off[p] * r.dp, st));
    }
    return CIQ_OK;
}

template <typename T>
void fill_problem_tables(Run<T>& r, const ciq_problem* probs, int nprob, int dtype) {
    r.dtype = dtype;
    r.nprob = nprob;
    r.h_n.resize(nprob);
    r.h_off.resize(nprob);
    r.h_o2.resize(nprob);
    r.h_s2.resize(nprob);
    r.h_o2d.resize(nprob);
    r.h_s2d.resize(nprob);
    int off = 0, maxn = 0, maxd = 1;
    for (int p = 0; p < nprob; ++p) {
        r.h_n[p] = probs[p].n;
        r.h_off[p] = off;
        off += probs[p].n;
        maxn = std::max(maxn, probs[p].n);
        maxd = std::max(maxd, probs[p].d);
        r.h_o2[p] = (float)probs[p].outputscale;
        r.h_s2[p] = (float)probs[p].noise;
        r.h_o2d[p] = probs[p].outputscale;
        r.h_s2d[p] = probs[p].noise;
    }
    r.h_scale.assign((size_t)nprob * CIQ_MAX_D, 0.0);
    r.ard = 0;
    for (int p = 0; p < nprob; ++p) {
        double sc[CIQ_MAX_D];
        point_scale(&probs[p], dtype, sc);
        for (int k = 0; k < probs[p].d; ++k) {
            r.h_scale[(size_t)p * CIQ_MAX_D + k] = sc[k];
            if (sc[k] != sc[0]) r.ard = 1;
        }
    }
    r.rows_total = off;
    r.max_n = maxn;
    // resident matrices one after another (FP32 elements), each in its own padded layout
    r.h_pkt.resize(nprob);
    r.h_pnjs.resize(nprob);
    long long kofs = 0;
    for (int p = 0; p < nprob; ++p) {
        r.h_pkt[p] = kofs;
        r.h_pnjs[p] = (long long)(kcache_cols(probs[p].n) / 4);
        kofs += (long long)(kcache_rows(probs[p].n) * kcache_cols(probs[p].n));
    }
    r.dp = pad_dims(maxd, r.dtype);
    r.kernel = probs[0].kernel;
}

// Resident kernel matrix of one call: allocated after the decision in solve(),
// freed when the call returns (after the device has drained its work).
struct KCache {
    void* ptr = nullptr;
    int elem = 8;
    ~KCache() {
        if (ptr) {
            (void)hipDeviceSynchronize();
            (void)hipFree(ptr);
        }
    }
};

// Whether (and then where) a solve keeps K resident; CIQ_OK with *out = nullptr
// means the products evaluate entries on the fly.
int kcache_acquire(const ciq_opts* o, int dtype, int nprob, const ciq_problem* probs, KCache& kc) {
    if ((dtype != CIQ_F64 && dtype != CIQ_F32 && dtype != CIQ_F16X3) || o->kernel_cache == CIQ_CACHE_OFF)
        return CIQ_OK;
    if (nprob != 1 && dtype != CIQ_F32) return CIQ_OK;   // batched: FP32 matrices, one per problem
    kc.elem = (dtype == CIQ_F64) ? 8 : 4;    // FP32, or the FP16 hi + lo pair
    size_t bytes = 0;
    for (int p = 0; p < nprob; ++p) bytes += kcache_bytes(probs[p].n, kc.elem);
    if (o->kernel_cache != CIQ_CACHE_ON) {
        size_t fr = 0, tot = 0;
        HIPCHK(hipMemGetInfo(&fr, &tot));
        if (bytes > fr / 2) {   // basis chunks kept from earlier calls give way to the matrix
            int dev = 0;
            HIPCHK(hipGetDevice(&dev));
            if (!g_basis[dev].chunks.empty()) {
                STCHK(basis_pool_release(dev));
                HIPCHK(hipMemGetInfo(&fr, &tot));
            }
        }
        size_t limit = fr / 2;
        if (o->cache_budget_mib > 0) limit = std::min(limit, (size_t)o->cache_budget_mib << 20);
        if (bytes > limit) return CIQ_OK;
    }
    if (!dev_malloc(&kc.ptr, bytes)) {
        (void)hipGetLastError();
        kc.ptr = nullptr;
        return o->kernel_cache == CIQ_CACHE_ON ? CIQ_ENOMEM : CIQ_OK;
    }
    return CIQ_OK;
}

// Writes the resident matrix for the single problem of r and points r's
// products at it.
template <typename T>
int kcache_build(Run<T>& r, const KCache& kc, hipStream_t st) {
    if (!kc.ptr) return CIQ_OK;
    if (r.nprob > 1) {   // one FP32 matrix per problem, entries in FP64 rounded once
        for (int p = 0; p < r.nprob; ++p) {
            KBuildArgs ka{};
            ka.xh = r.xh + (size_t)r.h_off[p] * r.dp;
            ka.ard = 0;
            for (int k = 0; k < CIQ_MAX_D; ++k) {
                ka.scale[k] = r.h_scale[(size_t)p * CIQ_MAX_D + k];
                if (ka.scale[k] != ka.scale[0] && ka.scale[k] != 0.0) ka.ard = 1;
            }
            ka.n = r.h_n[p];
            ka.dp = r.dp;
            ka.kernel = r.kernel;
            ka.nchunk = (int)(kcache_cols(ka.n) / 64);
            ka.njs = (long long)(kcache_cols(ka.n) / 4);
            ka.elem = 1;
            ka.kt = static_cast<float*>(kc.ptr) + r.h_pkt[p];
            HIPCHK(launch_kbuild(ka, st));
        }
        r.kt = kc.ptr;
        return CIQ_OK;
    }
    KBuildArgs ka{};
    ka.xh = r.xh;
    for (int k = 0; k < CIQ_MAX_D; ++k) ka.scale[k] = r.h_scale[k];
    ka.n = r.h_n[0];
    ka.dp = r.dp;
    ka.kernel = r.kernel;
    ka.ard = r.ard;
    ka.nchunk = (int)(kcache_cols(ka.n) / 64);
    ka.njs = (long long)(kcache_cols(ka.n) / 4);
    ka.elem = (r.dtype == CIQ_F16X3) ? 2 : (kc.elem == 4 ? 1 : 0);
    ka.kt = kc.ptr;
    HIPCHK(launch_kbuild(ka, st));
    r.kt = kc.ptr;
    r.njs = ka.njs;
    return CIQ_OK;
}

struct ScratchLock {
    std::unique_lock<std::mutex> lk;
    explicit ScratchLock(int dev) : lk(g_scratch[dev].mu) {}
};

// Full CIQ solve for nprob problems sharing s, Q, dtype, kernel.
// out_ptrs[p]: n_p x s with leading dimension ldo; b_ptrs likewise with ldb.
template <typename T>
int solve(int nprob, const ciq_problem* probs, const ciq_opts* o, const void* const* b_ptrs, int s, int ldb,
          void* const* out_ptrs, int ldo, void* solves_out, int mode, ciq_info* infos, hipStream_t st,
          const PostSpec* post_spec = nullptr, const SparseOp* sparse = nullptr, const DenseOp* dense = nullptr) {
    int dev;
    STCHK(get_device(&dev));
    ScratchLock lock(dev);
    const int dtype = o->dtype;
    const int check_every = o->check_every > 0 ? o->check_every : 16;
    const int steps = o->lanczos_steps > 0 ? o->lanczos_steps : 20;
    // a dense operator means one plain solve (shift 0, weight 1): no bounds
    const bool have_bounds = dense != nullptr || (o->lambda_min > 0.0 && o->lambda_max >= o->lambda_min &&
                                                  std::isfinite(o->lambda_max));
    const bool profile = o->profile != 0;

    KCache kc;
    if (!sparse && !dense) STCHK(kcache_acquire(o, dtype, nprob, probs, kc));
    const bool precond = o->precond_rank > 0;
    Precond pc;
    Posterior po;

    // ---- sizing: bounds run (s = 1, Q = 0) and main run share the points ----
    Run<T> main;
    fill_problem_tables(main, probs, nprob, dtype);
    main.cached = (kc.ptr != nullptr);
    main.precond = precond;
    main.sp = sparse;
    main.dn = dense;
    main.dtype = dtype;
    main.s = s;
    main.Q = o->q;
    main.max_iter = o->max_iter;
    main.tol = o->tol;
    main.keep_solves = (solves_out != nullptr);
    // the inverse root amplifies the products' FP32 rounding in the
    // noise-level eigendirections; the square root's final K damps it
    main.fine_acc = (mode != CIQ_SQRT) ? 1 : 0;
    // likewise the square root's resident FP32 / split-FP16 products leave
    // their column-range partials in FP32 (one rounding each, below that of
    // the FP32 chunk sums inside them), halving what the reduction reads;
    // the inverse root keeps FP64 partials
    main.part32 = (mode == CIQ_SQRT) && nprob == 1 && main.cached && (dtype == CIQ_F32 || dtype == CIQ_F16X3) &&
                  !precond && post_spec == nullptr && sparse == nullptr && dense == nullptr;
    main.plan(2);

    Run<T> bnd;
    fill_problem_tables(bnd, probs, nprob, dtype);
    bnd.dtype = dtype;
    bnd.s = 1;
    bnd.Q = 0;
    bnd.max_iter = steps;
    bnd.tol = 0.0;
    bnd.bounds_mode = 1;
    bnd.cached = main.cached;
    bnd.precond = precond;
    bnd.sp = sparse;
    bnd.dn = dense;
    bnd.plan(2);

    Sizer sz;
    main.layout(sz, true);
    const size_t off_after_xh = 0;
    (void)off_after_xh;
    Sizer szb;
    szb.take<double>((size_t)main.rows_total * main.dp);
    bnd.layout(szb, false);
    const size_t need = std::max(sz.off, szb.off) + 4096;
    void* base = nullptr;
    STCHK(scratch_reserve(dev, need, &base));
    IterState* pinned = g_scratch[dev].pinned;

    Carver cm(base);
    main.layout(cm, true);
    Carver cb(base);
    bnd.xh = cb.take<double>((size_t)main.rows_total * main.dp);
    bnd.layout(cb, false);
    main.fill_dev();
    bnd.fill_dev();

    STCHK(main.upload_tables(st));
    if (!sparse && !dense) STCHK(setup_points(main, probs, dtype, st));
    STCHK(kcache_build(main, kc, st));
    bnd.kt = main.kt;
    bnd.njs = main.njs;
    // the point and matrix set-up above is queued work: finish it first so
    // the factors' build time is their own
    if (precond || post_spec) HIPCHK(hipStreamSynchronize(st));
    const auto setup_t0 = std::chrono::steady_clock::now();
    if (precond) {
        STCHK(pc_build(probs[0], main.xh, main.dp, main.kernel, main.ard, main.h_scale.data(), o->precond_rank, s,
                       pc, st));
        main.pc = &pc;
        bnd.pc = &pc;
        // the operand p_j = P^{-1} z_j has p_j^T z_j = 1 and P >= sigma^2 I, so
        // |p_j| <= 1/sigma: scale it by the power of two at most 256 sigma
        const float sc = (float)std::ldexp(1.0, (int)std::floor(std::log2(256.0 * std::sqrt(probs[0].noise))));
        main.op_scale = sc;
        bnd.op_scale = sc;
    }
    if (post_spec) {
        STCHK(post_build(probs[0], dtype, main.xh, main.dp, main.kernel, main.ard, main.h_scale.data(), *post_spec,
                         s, po, st));
        main.post = &po;
        bnd.post = &po;
    }
    // both builds end synchronised with the stream
    const double setup_ms = (precond || post_spec)
        ? std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - setup_t0).count()
        : 0.0;

    std::vector<double> lmin(nprob), lmax(nprob);
    int mvm_count = 0;
    double mvm_ms = 0.0;
    int mvm_timed = 0;
    std::vector<hipEvent_t> evs;
    if (profile) {
        evs.resize(2 * check_every);
        for (auto& e : evs) HIPCHK(hipEventCreate(&e));
    }
    struct EvGuard {
        std::vector<hipEvent_t>& v;
        ~EvGuard() {
            for (auto e : v) (void)hipEventDestroy(e);
        }
    } evguard{evs};

    if (have_bounds) {
        for (int p = 0; p < nprob; ++p) {
            lmin[p] = o->lambda_min;
            lmax[p] = o->lambda_max;
        }
    } else {
        STCHK(bnd.upload_tables(st));
        for (int p = 0; p < nprob; ++p)
            HIPCHK(launch_splitmix<double>(bnd.qbuf[0] + bnd.h_off[p], bnd.h_n[p], o->seed + 7919ull * p, 1, st));
        int cnt = 0, dummy_n = 0;
        double dummy = 0.0;
        STCHK(bnd.iterate(st, std::max(steps, 1), pinned, &cnt, nullptr, 0, &dummy, &dummy_n));
        mvm_count += cnt;
        const int J = pinned->iter;
        std::vector<double> Th((size_t)std::max(J, 1) * nprob * 2);
        if (J > 0)
            HIPCHK(hipMemcpyAsync(Th.data(), bnd.d.T, Th.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        std::vector<int> citers(nprob);
        HIPCHK(hipMemcpyAsync(citers.data(), bnd.d.col_iters, nprob * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int p = 0; p < nprob; ++p) {
            const int Jp = std::max(1, citers[p]);
            std::vector<double> al(Jp), be(Jp);
            for (int j = 0; j < Jp; ++j) {
                al[j] = Th[((size_t)j * nprob + p) * 2 + 0];
                be[j] = Th[((size_t)j * nprob + p) * 2 + 1];
            }
            // floor of the spectrum: sigma^2 for K, 1 for P^{-1/2} K P^{-1/2}
            bounds_from_tridiag(Jp, al.data(), be.data(), precond ? 1.0 : probs[p].noise, &lmin[p], &lmax[p]);
            if (!(lmin[p] > 0.0) || !(lmax[p] >= lmin[p]) || !std::isfinite(lmax[p])) return CIQ_ENUMERIC;
        }
        // the bounds run reused the scratch after the points; restore the main tables
        STCHK(main.upload_tables(st));
    }

    // ---- shifts / weights --------------------------------------------------
    std::vector<double> th((size_t)nprob * main.Q), wh((size_t)nprob * main.Q);
    for (int p = 0; p < nprob; ++p) {
        if (dense) {                       // x = A^{-1} b: one shift t = 0 of weight 1
            for (int q = 0; q < main.Q; ++q) {
                th[(size_t)p * main.Q + q] = 0.0;
                wh[(size_t)p * main.Q + q] = (q == 0) ? 1.0 : 0.0;
            }
            continue;
        }
        const int rc = ciq_setup(lmin[p], lmax[p], main.Q, &th[(size_t)p * main.Q], &wh[(size_t)p * main.Q]);
        if (rc != CIQ_OK) return CIQ_ENUMERIC;
    }
    HIPCHK(hipMemcpyAsync(main.t, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(main.w, wh.data(), wh.size() * sizeof(double), hipMemcpyHostToDevice, st));

    // ---- right-hand sides --------------------------------------------------
    for (int p = 0; p < nprob; ++p)
        HIPCHK((launch_copy<T, double>(static_cast<const T*>(b_ptrs[p]), ldb, main.h_n[p], s,
                                       main.qbuf[0] + (size_t)main.h_off[p] * s, s, st)));
    HIPCHK(hipStreamSynchronize(st));  // th/wh are pageable host vectors
    if (precond)   // start vectors C = P^{1/2} B (Appendix D), in place
        STCHK(pc_apply(pc, std::sqrt(pc.s2), pc.fsq, main.qbuf[0], main.rows_total, s, main.qbuf[0], nullptr, nullptr,
                       nullptr, st));
    if (main.q32) {
        HIPCHK((launch_copy<double, float>(main.qbuf[0], s, main.rows_total, s, main.q32, s, st)));
        STCHK(tune_rt(main, main.q32, st));
    } else {
        if (main.vt16)   // the trial launches read the split operand: give them zeros
            HIPCHK(launch_fill<int>(static_cast<int*>(main.vt16), op16_halfs(kcache_cols(main.max_n), main.nsbt) / 2,
                                    0, st));
        STCHK(tune_rt(main, main.qbuf[0], st));
    }

    // ---- resident Krylov basis (when every slot the run may reach fits) -----
    BasisSlots bslots;
    double *basis_cq = nullptr, *basis_c = nullptr;
    bool use_basis = false;
    if (o->krylov_basis == CIQ_BASIS_AUTO && !precond && solves_out == nullptr && main.Q > 0) {
        BasisPool& bp = g_basis[dev];
        const size_t slots = (size_t)main.max_iter + 1;
        const size_t stride = ((size_t)main.rows_total * s * sizeof(double) + 255) & ~size_t(255);
        const size_t chunk = basis_chunk_bytes(stride);
        if (bp.chunk_bytes != chunk) {   // another chunk size: start the pool over
            STCHK(basis_pool_release(dev));
            bp.chunk_bytes = chunk;
        }
        const size_t per_chunk = chunk / stride;
        const size_t chunks = (slots + per_chunk - 1) / per_chunk;
        const size_t qn = (size_t)main.Q * main.d.ncol;
        const size_t iters_cap = (size_t)main.max_iter;
        auto log_layout = [&](auto& c) {   // coefficient logs and the slot table
            main.d.clog = c.template take<double>(iters_cap * qn * 4);
            basis_cq = c.template take<double>(iters_cap * qn);
            basis_c = c.template take<double>(iters_cap * main.d.ncol);
            bslots.tab = c.template take<double*>(slots);
        };
        Sizer lz;
        log_layout(lz);
        const size_t logs = lz.off;
        const size_t more =
            (chunks > bp.chunks.size() ? (chunks - bp.chunks.size()) * chunk : 0) + (logs > bp.logs_cap ? logs : 0);
        bool fits = true;
        if (more > 0) {   // leave a tenth of the free memory and 4 GiB for everything else
            size_t free_b = 0, total_b = 0;
            fits = hipMemGetInfo(&free_b, &total_b) == hipSuccess && more + (size_t(4) << 30) <= free_b / 10 * 9;
            if (!fits) (void)hipGetLastError();
        }
        if (fits && logs > bp.logs_cap) {
            if (bp.logs) {
                HIPCHK(hipDeviceSynchronize());
                HIPCHK(hipFree(bp.logs));
                bp.logs = nullptr;
                bp.logs_cap = 0;
            }
            if (hipMalloc(&bp.logs, logs) == hipSuccess) {
                bp.logs_cap = logs;
            } else {
                (void)hipGetLastError();
                bp.logs = nullptr;
                fits = false;
            }
        }
        if (fits) {
            Carver lc(bp.logs);
            log_layout(lc);
            bslots.dev = dev;
            bslots.stride = stride;
            bslots.per_chunk = (int)per_chunk;
            bslots.max_slots = (int)slots;
            HIPCHK(launch_fill<double>(reinterpret_cast<double*>(bslots.tab), slots, 0.0, st));   // null pointers
            // the pooled chunks at once; the run takes new ones as it reaches them
            STCHK(bslots.ensure((int)std::min(bp.chunks.size() * per_chunk, slots), st));
            main.d.basis = bslots.tab;
            main.d.basis_slots = (int)slots;
            main.bslots = &bslots;
            use_basis = true;
        } else {
            main.d.clog = nullptr;
            basis_cq = basis_c = nullptr;
            bslots.tab = nullptr;
        }
    }

    STCHK(main.iterate(st, check_every, pinned, &mvm_count, profile ? evs.data() : nullptr,
                       profile ? check_every : 0, &mvm_ms, &mvm_timed, o->graph == 1));
    const int iters = pinned->iter;
    if (use_basis && iters > 0)
        HIPCHK(launch_basis_combine(main.d, iters, basis_cq, basis_c, main.acc, main.max_n, st));

    // ---- combine -----------------------------------------------------------
    if (mode == CIQ_SQRT) {
        const void* operand = main.acc;
        if (main.q32) {
            HIPCHK((launch_copy<double, float>(main.acc, s, main.rows_total, s, main.q32, s, st)));
            operand = main.q32;
        }
        if (main.vt16)   // the combined solution is not unit-norm: per-column scales
            HIPCHK(launch_op16_split(main.acc, main.rows_total, s, s, main.opsc, main.opinv, main.vt16, main.nsbt,
                                     st));
        MvmArgs a = main.mvm_args(operand, main.ypart);
        a.done = nullptr;
        a.prob_done = nullptr;
        if (main.vt16) a.vcol_inv = main.opinv;
        if (sparse)
            HIPCHK(launch_spmv(*sparse, main.acc, s, s, main.ypart, s, nullptr, st));
        else if (dense)
            HIPCHK(launch_lr_apply(0.0, nullptr, 0, dense->A, dense->n, main.acc, s, main.rows_total, dense->n, s,
                                   main.ypart, s, nullptr, nullptr, nullptr, st));
        else
            HIPCHK(launch_mvm(dtype, a, st));
        STCHK(main.post_correct(main.acc, nullptr, st));
        mvm_count += 1;
        for (int p = 0; p < nprob; ++p)
            HIPCHK(launch_reduce_splits<T>(main.ypart + (size_t)main.h_off[p] * s, main.ysplit, main.nsplit, s,
                                           main.h_n[p], s, static_cast<T*>(out_ptrs[p]), ldo, st));
    } else {
        for (int p = 0; p < nprob; ++p)
            HIPCHK((launch_copy<double, T>(main.acc + (size_t)main.h_off[p] * s, s, main.h_n[p], s,
                                           static_cast<T*>(out_ptrs[p]), ldo, st)));
    }
    if (solves_out) {
        HIPCHK((launch_copy<double, T>(main.solves, s, main.rows_total * main.Q, s, static_cast<T*>(solves_out),
                                       s, st)));
    }

    // ---- report ------------------------------------------------------------
    const int ncol = nprob * s;
    const size_t qn = (size_t)main.Q * ncol;
    std::vector<int> frozen(qn), citers(ncol);
    std::vector<double> relres(qn);
    if (qn) {
        HIPCHK(hipMemcpyAsync(frozen.data(), main.d.frozen, qn * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(relres.data(), main.d.relres, qn * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(citers.data(), main.d.col_iters, ncol * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int p = 0; p < nprob; ++p) {
        ciq_info& in = infos[p];
        std::memset(&in, 0, sizeof(in));
        int it = 0, conv = 1;
        double mr = 0.0;
        for (int c = 0; c < s; ++c) {
            const int g = p * s + c;
            it = std::max(it, citers[g]);
            for (int q = 0; q < main.Q; ++q) {
                const size_t idx = (size_t)q * ncol + g;
                mr = std::max(mr, relres[idx]);
                if (!(relres[idx] <= main.tol)) conv = 0;
            }
        }
        in.iters = (nprob == 1) ? iters : it;
        in.converged = conv;
        in.q = main.Q;
        in.mvm_count = mvm_count;
        in.max_rel_residual = mr;
        in.lambda_min = lmin[p];
        in.lambda_max = lmax[p];
        for (int q = 0; q < main.Q; ++q) {
            in.t[q] = th[(size_t)p * main.Q + q];
            in.w[q] = wh[(size_t)p * main.Q + q];
        }
        in.mvm_ms = mvm_ms;
        in.mvm_timed = mvm_timed;
        in.kernel_cached = (kc.ptr != nullptr) ? 1 : 0;
        in.precond_rank = precond ? pc.rank : 0;
        in.precond_trace = precond ? pc.trace : 0.0;
        in.setup_ms = setup_ms;
        in.krylov_basis = use_basis ? 1 : 0;
    }
    return CIQ_OK;
}

int check_solve_args(const ciq_problem* p, const ciq_opts* o, const void* b, int s, int ldb, void* out,
                     int ldo, ciq_info* info) {
    if (!valid_problem(p) || !o || !b || !out || !info) return CIQ_EINVAL;
    if (!valid_dtype(o->dtype)) return CIQ_EINVAL;
    if (s < 1 || ldb < s || ldo < s) return CIQ_EINVAL;
    if (o->q < 1 || o->q > CIQ_MAX_Q || o->max_iter < 1) return CIQ_EINVAL;
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return CIQ_EINVAL;
    if (o->lanczos_steps < 0 || o->check_every < 0) return CIQ_EINVAL;
    if (o->krylov_basis != CIQ_BASIS_AUTO && o->krylov_basis != CIQ_BASIS_OFF) return CIQ_EINVAL;
    if (o->precond_rank < 0 || o->precond_rank > CIQ_MAX_RANK) return CIQ_EINVAL;
    if (o->precond_rank > 0 && !(p->noise > 0.0)) return CIQ_EINVAL;   // P = Lbar Lbar^T + sigma^2 I
    return CIQ_OK;
}

// Backward of a forward call (Sec. 3.3): one msMINRES run on G' = G (inverse
// root) or K G (root) with the forward's shifts, dB = sum_q w_q g_q, then the
// tile pass contracting W = sum_q w_q g_q a_q^T (+ the root's direct term)
// with dK/dtheta.
template <typename T>
int backward_impl(const ciq_problem* p, const ciq_opts* o, int mode, const double* t, const double* w,
                  const void* solves, const void* g, int s, int ldg, void* db, int lddb, double* dls,
                  double* do2, double* dnoise, ciq_info* info, hipStream_t st) {
    int dev;
    STCHK(get_device(&dev));
    ScratchLock lock(dev);
    const int dtype = o->dtype;
    const int Q = o->q;
    const int n = p->n;
    const bool sqrt_mode = (mode == CIQ_SQRT);
    const bool want_hyper = dls || do2 || dnoise;

    KCache kc;
    STCHK(kcache_acquire(o, dtype, 1, p, kc));
    Run<T> r;
    fill_problem_tables(r, p, 1, dtype);
    r.dtype = dtype;
    r.s = s;
    r.Q = Q;
    r.max_iter = o->max_iter;
    r.tol = o->tol;
    r.keep_solves = true;
    r.fine_acc = sqrt_mode ? 0 : 1;
    r.cached = (kc.ptr != nullptr);
    r.plan(2);

    const int kpad = grad_k_pad((Q + (sqrt_mode ? 1 : 0)) * s);
    const int rows_pad = grad_rows_pad(n);
    const int dpg = pad_dims(p->d, -1);   // gradient pass instantiations
    const int nb = rows_pad / 64;
    auto extra = [&](auto& a, double** U, double** V, double** pts, double** xd, double** part) {
        *U = a.template take<double>(want_hyper ? (size_t)rows_pad * kpad : 1);
        *V = a.template take<double>(want_hyper ? (size_t)rows_pad * kpad : 1);
        *pts = a.template take<double>((size_t)n * dpg);
        *xd = a.template take<double>((size_t)n * p->d);
        *part = a.template take<double>((size_t)nb * nb * (dpg + 2));
    };
    double *U, *V, *pts, *xd, *part;
    Sizer sz;
    r.layout(sz, true);
    extra(sz, &U, &V, &pts, &xd, &part);
    void* base = nullptr;
    STCHK(scratch_reserve(dev, sz.off + 4096, &base));
    IterState* pinned = g_scratch[dev].pinned;
    Carver c(base);
    r.layout(c, true);
    extra(c, &U, &V, &pts, &xd, &part);
    r.fill_dev();
    STCHK(r.upload_tables(st));
    STCHK(setup_points(r, p, dtype, st));
    STCHK(kcache_build(r, kc, st));
    HIPCHK(hipMemcpyAsync(r.t, t, Q * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(r.w, w, Q * sizeof(double), hipMemcpyHostToDevice, st));

    // G' into the first Lanczos buffer (FP64)
    if (sqrt_mode) {
        MvmArgs a = r.mvm_args(g, r.ypart);
        a.ldv = ldg;
        a.done = nullptr;
        HIPCHK(launch_mvm(dtype, a, st));
        HIPCHK(launch_reduce_splits<double>(r.ypart, r.ysplit, r.nsplit, s, n, s, r.qbuf[0], s, st));
    } else {
        HIPCHK((launch_copy<T, double>(static_cast<const T*>(g), ldg, n, s, r.qbuf[0], s, st)));
    }
    HIPCHK(hipStreamSynchronize(st));   // t/w came from caller-owned host memory
    int mvm_count = sqrt_mode ? 1 : 0, dummy_n = 0;
    double dummy = 0.0;
    STCHK(r.iterate(st, o->check_every > 0 ? o->check_every : 16, pinned, &mvm_count, nullptr, 0, &dummy,
                    &dummy_n));
    const int iters = pinned->iter;
    if (db) HIPCHK((launch_copy<double, T>(r.acc, s, n, s, static_cast<T*>(db), lddb, st)));

    double acc_h[CIQ_MAX_D + 2] = {0};
    if (want_hyper) {
        // points scaled by 1/l per dimension, in FP64
        HIPCHK((launch_copy<T, double>(static_cast<const T*>(p->x), p->d, n, p->d, xd, p->d, st)));
        double scale[CIQ_MAX_D];
        for (int k = 0; k < p->d; ++k) scale[k] = 1.0 / p->lengthscale[p->n_lengthscale == 1 ? 0 : k];
        HIPCHK(launch_prep<double>(xd, n, p->d, dpg, scale, pts, st));
        HIPCHK(launch_build_uv<T>(r.solves, static_cast<const T*>(solves), static_cast<const T*>(g), ldg, r.w, n,
                                  Q, s, sqrt_mode ? 1 : 0, U, V, st));
        int nblocks = 0;
        HIPCHK(launch_grad_pass(p->kernel, U, V, kpad, pts, n, dpg, part, &nblocks, st));
        std::vector<double> hp((size_t)nblocks * (dpg + 2));
        HIPCHK(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int b = 0; b < nblocks; ++b)
            for (int k = 0; k < dpg + 2; ++k) acc_h[k] += hp[(size_t)b * (dpg + 2) + k];
    }
    // report of the backward msMINRES run
    const size_t qn = (size_t)Q * s;
    std::vector<double> relres(qn);
    HIPCHK(hipMemcpyAsync(relres.data(), r.d.relres, qn * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memset(info, 0, sizeof(*info));
    double mr = 0.0;
    int conv = 1;
    for (double v : relres) {
        mr = std::max(mr, v);
        if (!(v <= o->tol)) conv = 0;
    }
    info->iters = iters;
    info->converged = conv;
    info->q = Q;
    info->mvm_count = mvm_count;
    info->max_rel_residual = mr;
    info->kernel_cached = (kc.ptr != nullptr) ? 1 : 0;
    for (int q = 0; q < Q; ++q) {
        info->t[q] = t[q];
        info->w[q] = w[q];
    }
    if (want_hyper) {
        const double o2 = p->outputscale;
        if (dls) {
            if (p->n_lengthscale == 1) {
                double sum = 0.0;
                for (int k = 0; k < p->d; ++k) sum += acc_h[k];
                dls[0] = -o2 * sum / p->lengthscale[0];
            } else {
                for (int k = 0; k < p->d; ++k) dls[k] = -o2 * acc_h[k] / p->lengthscale[k];
            }
        }
        if (do2) *do2 = -acc_h[dpg];
        if (dnoise) *dnoise = -acc_h[dpg + 1];
    }
    return CIQ_OK;
}

// ---- on-the-fly kernel product (ciq_kernel_mvm and its allocation-free form)
struct KmvmPlan {
    int dp, nrb, nsplit;
    bool direct;            // FP64 into y directly (one split, <= 64 columns)
    size_t xbytes, ybytes;  // scaled points (256-byte rounded), FP64 split partials
};

KmvmPlan kmvm_plan(const ciq_problem* p, int dtype, int s) {
    KmvmPlan pl{};
    pl.dp = pad_dims(p->d, dtype);
    const int rpb = mvm_rows_per_block(dtype, s, 2);
    pl.nrb = (p->n + rpb - 1) / rpb;
    pl.nsplit = mvm_pick_nsplit(dtype, pl.nrb, p->n, s);
    pl.xbytes = ((size_t)p->n * pl.dp * sizeof(double) + 255) & ~size_t(255);
    pl.direct = (dtype == CIQ_F64 && pl.nsplit == 1 && s <= 64);
    pl.ybytes = pl.direct ? 0 : (size_t)pl.nsplit * p->n * s * sizeof(double);
    return pl;
}

// Queues Y = K V on `stream` with `buf` (>= xbytes + ybytes, 256-byte aligned)
// holding the scaled points and the split partials.
int kmvm_run(const ciq_problem* p, int dtype, const void* v, int s, int ldv, void* y, int ldy, const KmvmPlan& pl,
             void* buf, hipStream_t stream) {
    double scale[CIQ_MAX_D];
    point_scale(p, dtype, scale);
    double ones[CIQ_MAX_D];
    for (int k = 0; k < CIQ_MAX_D; ++k) ones[k] = 1.0;
    hipError_t e;
    if (dtype == CIQ_F64)
        e = launch_prep<double>(static_cast<const double*>(p->x), p->n, p->d, pl.dp, ones, static_cast<double*>(buf),
                                stream);
    else
        e = launch_prep<float>(static_cast<const float*>(p->x), p->n, p->d, pl.dp, ones, static_cast<double*>(buf),
                               stream);
    if (e != hipSuccess) return CIQ_EHIP;
    MvmArgs a{};
    a.xh = buf;
    a.v = v;
    a.y = pl.direct ? y : static_cast<void*>(static_cast<char*>(buf) + pl.xbytes);
    a.ysplit = pl.direct ? 0 : (long long)p->n * s;
    a.ldv = ldv;
    a.ldy = pl.direct ? ldy : s;
    a.s = s;
    a.kernel = p->kernel;
    a.dp = pl.dp;
    a.nsplit = pl.nsplit;
    a.rt = 2;
    a.ard = 0;
    for (int k = 0; k < CIQ_MAX_D; ++k) {
        a.scale[k] = (k < p->d) ? scale[k] : 0.0;
        if (k < p->d && scale[k] != scale[0]) a.ard = 1;
    }
    a.pscale = nullptr;
    a.n = p->n;
    a.o2 = p->outputscale;
    a.s2 = p->noise;
    a.nrb = pl.nrb;
    if (launch_mvm(dtype, a, stream) != hipSuccess) return CIQ_EHIP;
    if (!pl.direct) {
        if (dtype == CIQ_F64)
            e = launch_reduce_splits<double>(static_cast<const double*>(a.y), a.ysplit, pl.nsplit, s, p->n, s,
                                             static_cast<double*>(y), ldy, stream);
        else
            e = launch_reduce_splits<float>(static_cast<const double*>(a.y), a.ysplit, pl.nsplit, s, p->n, s,
                                            static_cast<float*>(y), ldy, stream);
        if (e != hipSuccess) return CIQ_EHIP;
    }
    return CIQ_OK;
}

// Scratch of ciq_kernel_mvm_noalloc: a static device array (one copy per GPU,
// held until the process ends). Host code never passes `scratch` itself (on
// the host it names a stand-in, not device memory): its device address is
// taken once per device with hipGetSymbolAddress, with that device current,
// and only that address is used.
static __device__ __align__(256) unsigned char scratch[CIQ_NOALLOC_SCRATCH_BYTES];
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

int noalloc_scratch(int dev, void** out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return CIQ_EHIP;
        }
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return CIQ_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

int ciq_version(void) { return 100; }

const char* ciq_strerror(int status) {
    switch (status) {
        case CIQ_OK: return "CIQ_OK";
        case CIQ_EINVAL: return "CIQ_EINVAL: invalid argument";
        case CIQ_ENOMEM: return "CIQ_ENOMEM: device scratch allocation failed";
        case CIQ_EHIP: return "CIQ_EHIP: HIP runtime error";
        case CIQ_ENOTSUP: return "CIQ_ENOTSUP: not supported by this build";
        case CIQ_ENUMERIC: return "CIQ_ENUMERIC: non-finite Lanczos scalar";
        default: return "CIQ: unknown status";
    }
}

int ciq_release_workspace(int device) {
    if (device < 0 || device >= kMaxDevices) return CIQ_EINVAL;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device >= ndev) return CIQ_EINVAL;
    ScratchLock lock(device);
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != device) HIPCHK(hipSetDevice(device));
    int rc = basis_pool_release(device);
    DeviceScratch& sc = g_scratch[device];
    if (rc == CIQ_OK && sc.ptr) {
        if (hipDeviceSynchronize() != hipSuccess || hipFree(sc.ptr) != hipSuccess) rc = CIQ_EHIP;
        sc.ptr = nullptr;
        sc.cap = 0;
    }
    if (cur != device && hipSetDevice(cur) != hipSuccess && rc == CIQ_OK) rc = CIQ_EHIP;
    return rc;
}

int ciq_setup(double lambda_min, double lambda_max, int q, double* t_out, double* w_out) {
    if (!t_out || !w_out || q < 1 || q > CIQ_MAX_Q) return CIQ_EINVAL;
    if (!(lambda_min > 0.0) || !(lambda_max >= lambda_min) || !std::isfinite(lambda_max)) return CIQ_EINVAL;
    return ciq::hht_quadrature(lambda_min, lambda_max, q, t_out, w_out);
}

int ciq_kernel_mvm(const ciq_problem* p, int dtype, const void* v, int s, int ldv, void* y, int ldy,
                   hipStream_t stream) {
    if (!valid_problem(p) || !valid_dtype(dtype) || !v || !y || s < 1 || ldv < s || ldy < s) return CIQ_EINVAL;
    const KmvmPlan pl = kmvm_plan(p, dtype, s);
    // stream-ordered scratch: scaled points + FP64 split partials
    void* buf = nullptr;
    if (hipMallocAsync(&buf, pl.xbytes + pl.ybytes, stream) != hipSuccess) {
        (void)hipGetLastError();
        return CIQ_ENOMEM;
    }
    const int rc = kmvm_run(p, dtype, v, s, ldv, y, ldy, pl, buf, stream);
    if (hipFreeAsync(buf, stream) != hipSuccess) return CIQ_EHIP;
    return rc;
}

int ciq_kernel_mvm_noalloc(const ciq_problem* p, int dtype, const void* v, int s, int ldv, void* y, int ldy,
                           hipStream_t stream) {
    if (!valid_problem(p) || !valid_dtype(dtype) || !v || !y || s < 1 || ldv < s || ldy < s) return CIQ_EINVAL;
    const KmvmPlan pl = kmvm_plan(p, dtype, s);
    if (pl.xbytes + pl.ybytes > (size_t)CIQ_NOALLOC_SCRATCH_BYTES) return CIQ_EINVAL;
    int dev;
    STCHK(get_device(&dev));
    void* buf = nullptr;
    STCHK(noalloc_scratch(dev, &buf));
    return kmvm_run(p, dtype, v, s, ldv, y, ldy, pl, buf, stream);
}

int ciq_kernel_mvm_resident(const ciq_problem* p, int dtype, const void* v, int s, int ldv, void* y, int ldy,
                            hipStream_t stream) {
    if (!valid_problem(p) || !valid_dtype(dtype) || !v || !y || s < 1 || ldv < s || ldy < s) return CIQ_EINVAL;
    if (dtype == CIQ_BF16X3) return CIQ_ENOTSUP;
    int dev;
    STCHK(get_device(&dev));
    ScratchLock lock(dev);
    ciq_opts o{};
    o.dtype = dtype;
    o.kernel_cache = CIQ_CACHE_ON;
    KCache kc;
    STCHK(kcache_acquire(&o, dtype, 1, p, kc));
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        Run<T> r;
        fill_problem_tables(r, p, 1, dtype);
        r.dtype = dtype;
        r.s = s;
        r.Q = 0;
        r.max_iter = 1;
        r.cached = true;
        r.plan(2);
        Sizer sz;
        r.layout(sz, true);
        void* base = nullptr;
        STCHK(scratch_reserve(dev, sz.off + 4096, &base));
        Carver c(base);
        r.layout(c, true);
        r.fill_dev();
        STCHK(r.upload_tables(stream));
        STCHK(setup_points(r, p, dtype, stream));
        STCHK(kcache_build(r, kc, stream));
        HIPCHK((launch_copy<T, double>(static_cast<const T*>(v), ldv, p->n, s, r.qbuf[0], s, stream)));
        const void* operand = r.qbuf[0];
        if (r.q32) {
            HIPCHK((launch_copy<double, float>(r.qbuf[0], s, p->n, s, r.q32, s, stream)));
            operand = r.q32;
        }
        if (r.vt16) {
            HIPCHK(launch_fill<int>(static_cast<int*>(r.vt16), op16_halfs(kcache_cols(p->n), r.nsbt) / 2, 0, stream));
            HIPCHK(launch_op16_split(r.qbuf[0], p->n, s, s, r.opsc, r.opinv, r.vt16, r.nsbt, stream));
        }
        STCHK(tune_rt(r, operand, stream));
        MvmArgs a = r.mvm_args(operand, r.ypart);
        a.done = nullptr;
        a.prob_done = nullptr;
        if (r.vt16) a.vcol_inv = r.opinv;
        HIPCHK(launch_mvm(dtype, a, stream));
        HIPCHK(launch_reduce_splits<T>(r.ypart, r.ysplit, r.nsplit, s, p->n, s, static_cast<T*>(y), ldy, stream));
        HIPCHK(hipStreamSynchronize(stream));
        return CIQ_OK;
    };
    if (dtype == CIQ_F64) return run(double{});
    return run(float{});
}

int ciq_eig_bounds(const ciq_problem* p, int dtype, int steps, const void* v0, uint64_t seed,
                   double* lambda_min, double* lambda_max, hipStream_t stream) {
    if (!valid_problem(p) || !valid_dtype(dtype) || !lambda_min || !lambda_max || steps < 0) return CIQ_EINVAL;
    if (dtype == CIQ_BF16X3 || dtype == CIQ_F16X3) dtype = CIQ_F32;
    int dev;
    STCHK(get_device(&dev));
    ScratchLock lock(dev);
    const int J = steps > 0 ? steps : 20;
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        Run<T> r;
        fill_problem_tables(r, p, 1, dtype);
        r.dtype = dtype;
        r.s = 1;
        r.Q = 0;
        r.max_iter = J;
        r.bounds_mode = 1;
        r.plan(2);
        Sizer sz;
        r.layout(sz, true);
        void* base = nullptr;
        STCHK(scratch_reserve(dev, sz.off + 4096, &base));
        Carver c(base);
        r.layout(c, true);
        r.fill_dev();
        STCHK(r.upload_tables(stream));
        STCHK(setup_points(r, p, dtype, stream));
        if (v0)
            HIPCHK((launch_copy<T, double>(static_cast<const T*>(v0), 1, p->n, 1, r.qbuf[0], 1, stream)));
        else
            HIPCHK(launch_splitmix<double>(r.qbuf[0], p->n, seed, 1, stream));
        int cnt = 0, dummy_n = 0;
        double dummy = 0.0;
        IterState* pinned = g_scratch[dev].pinned;
        STCHK(r.iterate(stream, J, pinned, &cnt, nullptr, 0, &dummy, &dummy_n));
        int Jp = 0;
        HIPCHK(hipMemcpy(&Jp, r.d.col_iters, sizeof(int), hipMemcpyDeviceToHost));
        Jp = std::max(Jp, 1);
        std::vector<double> Th((size_t)Jp * 2);
        HIPCHK(hipMemcpy(Th.data(), r.d.T, Th.size() * sizeof(double), hipMemcpyDeviceToHost));
        std::vector<double> al(Jp), be(Jp);
        for (int j = 0; j < Jp; ++j) {
            al[j] = Th[2 * j];
            be[j] = Th[2 * j + 1];
        }
        bounds_from_tridiag(Jp, al.data(), be.data(), p->noise, lambda_min, lambda_max);
        return CIQ_OK;
    };
    if (dtype == CIQ_F64) return run(double{});
    return run(float{});
}

static int solve_single(const ciq_problem* p, const ciq_opts* o, const void* b, int s, int ldb, void* out, int ldo,
                        void* solves, ciq_info* info, hipStream_t stream, int mode) {
    const int rc = check_solve_args(p, o, b, s, ldb, out, ldo, info);
    if (rc != CIQ_OK) return rc;
    const void* bp[1] = {b};
    void* op[1] = {out};
    if (o->dtype == CIQ_F64) return solve<double>(1, p, o, bp, s, ldb, op, ldo, solves, mode, info, stream);
    // F32 and the split forms: float inputs and outputs, FP64 vectors
    return solve<float>(1, p, o, bp, s, ldb, op, ldo, solves, mode, info, stream);
}

int ciq_invsqrt_mvm(const ciq_problem* p, const ciq_opts* o, const void* b, int s, int ldb, void* out, int ldo,
                    void* solves, ciq_info* info, hipStream_t stream) {
    return solve_single(p, o, b, s, ldb, out, ldo, solves, info, stream, CIQ_INVSQRT);
}

int ciq_sqrt_mvm(const ciq_problem* p, const ciq_opts* o, const void* b, int s, int ldb, void* out, int ldo,
                 void* solves, ciq_info* info, hipStream_t stream) {
    return solve_single(p, o, b, s, ldb, out, ldo, solves, info, stream, CIQ_SQRT);
}

int ciq_invsqrt_mvm_batched(int nprob, const ciq_problem* probs, const ciq_opts* o, const void* const* b, int s,
                            void* const* out, ciq_info* infos, hipStream_t stream) {
    if (nprob < 1 || !probs || !o || !b || !out || !infos || nprob > 1024) return CIQ_EINVAL;
    for (int p = 0; p < nprob; ++p) {
        const int rc = check_solve_args(&probs[p], o, b[p], s, s, out[p], s, &infos[p]);
        if (rc != CIQ_OK) return rc;
        if (probs[p].kernel != probs[0].kernel) return CIQ_EINVAL;
    }
    if (o->dtype != CIQ_F32 || o->precond_rank != 0) return CIQ_ENOTSUP;
    return solve<float>(nprob, probs, o, b, s, s, out, s, nullptr, CIQ_INVSQRT, infos, stream);
}

int ciq_backward(const ciq_problem* p, const ciq_opts* o, int mode, const double* t, const double* w,
                 const void* solves, const void* g, int s, int ldg, void* db, int lddb, double* dlengthscale,
                 double* doutputscale, double* dnoise, ciq_info* info, hipStream_t stream) {
    if (!valid_problem(p) || !o || !t || !w || !solves || !g || !info) return CIQ_EINVAL;
    if (!valid_dtype(o->dtype) || (mode != CIQ_INVSQRT && mode != CIQ_SQRT)) return CIQ_EINVAL;
    if (s < 1 || ldg < s || (db && lddb < s)) return CIQ_EINVAL;
    if (o->q < 1 || o->q > CIQ_MAX_Q || o->max_iter < 1 || !(o->tol >= 0.0) || !std::isfinite(o->tol))
        return CIQ_EINVAL;
    for (int q = 0; q < o->q; ++q)
        if (!(t[q] > 0.0) || !(w[q] > 0.0) || !std::isfinite(t[q]) || !std::isfinite(w[q])) return CIQ_EINVAL;
    if (o->precond_rank != 0) return CIQ_ENOTSUP;
    if (o->dtype == CIQ_F64)
        return backward_impl<double>(p, o, mode, t, w, solves, g, s, ldg, db, lddb, dlengthscale, doutputscale,
                                     dnoise, info, stream);
    if (o->dtype == CIQ_F32)
        return backward_impl<float>(p, o, mode, t, w, solves, g, s, ldg, db, lddb, dlengthscale, doutputscale,
                                    dnoise, info, stream);
    return CIQ_ENOTSUP;
}

int ciq_posterior_mvm(const ciq_problem* cand, const void* x_obs, int n_obs, double obs_noise, int mode,
                      const ciq_opts* o, const void* b, int s, int ldb, void* out, int ldo, ciq_info* info,
                      hipStream_t stream) {
    const int rc = check_solve_args(cand, o, b, s, ldb, out, ldo, info);
    if (rc != CIQ_OK) return rc;
    if (!x_obs || n_obs < 1 || n_obs > CIQ_MAX_OBS || !(obs_noise >= 0.0) || !std::isfinite(obs_noise))
        return CIQ_EINVAL;
    if (mode != CIQ_INVSQRT && mode != CIQ_SQRT) return CIQ_EINVAL;
    if (o->precond_rank != 0) return CIQ_ENOTSUP;
    const PostSpec ps{x_obs, n_obs, obs_noise};
    const void* bp[1] = {b};
    void* op[1] = {out};
    if (o->dtype == CIQ_F64) return solve<double>(1, cand, o, bp, s, ldb, op, ldo, nullptr, mode, info, stream, &ps);
    return solve<float>(1, cand, o, bp, s, ldb, op, ldo, nullptr, mode, info, stream, &ps);
}

int ciq_csr_mvm(const ciq_csr* a, int mode, const ciq_opts* o, const double* b, int s, int ldb, double* out,
                int ldo, ciq_info* info, hipStream_t stream) {
    if (!a || !a->row_ptr || !a->col_idx || !a->val || a->n < 1 || a->nnz < 0) return CIQ_EINVAL;
    if (mode != CIQ_INVSQRT && mode != CIQ_SQRT) return CIQ_EINVAL;
    // validate the options and sizes through the common check with a stand-in problem of n points
    const double one = 1.0;
    ciq_problem p{};
    p.n = a->n;
    p.d = 1;
    p.x = a->val;            // never read: the sparse operator replaces the kernel product
    p.kernel = CIQ_KERNEL_RBF;
    p.n_lengthscale = 1;
    p.lengthscale = &one;
    p.outputscale = 1.0;
    p.noise = 0.0;
    const int rc = check_solve_args(&p, o, b, s, ldb, out, ldo, info);
    if (rc != CIQ_OK) return rc;
    if (o->dtype != CIQ_F64 || o->precond_rank != 0) return CIQ_ENOTSUP;
    {   // the structure of the caller's CSR arrays, before any product reads them
        int dev;
        STCHK(get_device(&dev));
        ScratchLock lock(dev);
        void* base = nullptr;
        STCHK(scratch_reserve(dev, 4096, &base));
        int* bad = static_cast<int*>(base);
        HIPCHK(launch_fill<int>(bad, 1, 0, stream));
        HIPCHK(launch_csr_check(a->row_ptr, a->col_idx, a->n, a->nnz, bad, stream));
        int h_bad = 0;
        HIPCHK(hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        if (h_bad) return CIQ_EINVAL;
    }
    const SparseOp sp{a->n, a->row_ptr, a->col_idx, a->val};
    const void* bp[1] = {b};
    void* op[1] = {out};
    return solve<double>(1, &p, o, bp, s, ldb, op, ldo, nullptr, mode, info, stream, nullptr, &sp);
}

int ciq_svgp_predict(const ciq_problem* z, const void* x, int nb, const double* theta, const double* Theta,
                     const ciq_opts* o, int solve_max_iter, double solve_tol, double* mean, double* var,
                     double* a_out, ciq_info* info, ciq_info* info_solve, hipStream_t stream) {
    if (!valid_problem(z) || !o || !x || nb < 1 || !theta || !Theta || !mean || !var || !info) return CIQ_EINVAL;
    if (solve_max_iter < 1 || !(solve_tol >= 0.0) || !std::isfinite(solve_tol)) return CIQ_EINVAL;
    if (!valid_dtype(o->dtype)) return CIQ_EINVAL;
    if (o->dtype != CIQ_F64 && o->dtype != CIQ_F32) return CIQ_ENOTSUP;
    if (o->precond_rank != 0) return CIQ_ENOTSUP;
    const int M = z->n;
    const void* dummy_b = theta;   // shape checks only
    STCHK(check_solve_args(z, o, dummy_b, nb, nb, mean, nb, info));
    const int dp = pad_dims(z->d, CIQ_F64);
    double scale[CIQ_MAX_D], ones[CIQ_MAX_D];
    point_scale(z, o->dtype, scale);
    int ard = 0;
    for (int k = 0; k < CIQ_MAX_D; ++k) {
        ones[k] = 1.0;
        if (k >= z->d) scale[k] = 0.0;
        else if (scale[k] != scale[0]) ard = 1;
    }
    const bool f32 = (o->dtype == CIQ_F32);
    DevAlloc mem;
    size_t off = 0;
    double *xz = nullptr, *xx = nullptr, *kzx = nullptr, *a = nullptr, *thn = nullptr, *c = nullptr;
    float *k32 = nullptr, *a32 = nullptr;
    auto layout = [&](char* base) {
        off = 0;
        xz = carve<double>(base, off, (size_t)M * dp);
        xx = carve<double>(base, off, (size_t)nb * dp);
        kzx = carve<double>(base, off, (size_t)M * nb);
        a = carve<double>(base, off, (size_t)M * nb);
        c = carve<double>(base, off, (size_t)M * nb);
        thn = carve<double>(base, off, (size_t)M * M);
        if (f32) {
            k32 = carve<float>(base, off, (size_t)M * nb);
            a32 = carve<float>(base, off, (size_t)M * nb);
        }
    };
    layout(nullptr);
    if (!dev_malloc(&mem.p, off, false)) {   // no lock held here: the solves below take it
        (void)hipGetLastError();
        mem.p = nullptr;
        return CIQ_ENOMEM;
    }
    layout(static_cast<char*>(mem.p));
    hipError_t e;
    if (f32) {
        e = launch_prep<float>(static_cast<const float*>(z->x), M, z->d, dp, ones, xz, stream);
        if (e == hipSuccess) e = launch_prep<float>(static_cast<const float*>(x), nb, z->d, dp, ones, xx, stream);
    } else {
        e = launch_prep<double>(static_cast<const double*>(z->x), M, z->d, dp, ones, xz, stream);
        if (e == hipSuccess) e = launch_prep<double>(static_cast<const double*>(x), nb, z->d, dp, ones, xx, stream);
    }
    if (e != hipSuccess) return CIQ_EHIP;
    HIPCHK(launch_xkernel(xz, M, xx, nb, dp, z->kernel, ard, scale, z->outputscale, kzx, nb, stream));
    // a = Kzz^{-1/2} K_Zx by msMINRES-CIQ (Kzz with its jitter z->noise)
    if (f32) {
        HIPCHK((launch_copy<double, float>(kzx, nb, M, nb, k32, nb, stream)));
        const void* bp[1] = {k32};
        void* op[1] = {a32};
        STCHK(solve<float>(1, z, o, bp, nb, nb, op, nb, nullptr, CIQ_INVSQRT, info, stream));
        HIPCHK((launch_copy<float, double>(a32, nb, M, nb, a, nb, stream)));
    } else {
        const void* bp[1] = {kzx};
        void* op[1] = {a};
        STCHK(solve<double>(1, z, o, bp, nb, nb, op, nb, nullptr, CIQ_INVSQRT, info, stream));
    }
    // c = (-2 Theta)^{-1} a: MINRES on the dense operator (one shift 0, weight 1)
    HIPCHK(launch_scale(Theta, -2.0, thn, (long long)M * M, stream));
    ciq_opts so{};
    so.dtype = CIQ_F64;
    so.q = 1;
    so.max_iter = solve_max_iter;
    so.tol = solve_tol;
    so.check_every = o->check_every;
    const double one = 1.0;
    ciq_problem dp_{};
    dp_.n = M;
    dp_.d = 1;
    dp_.x = thn;             // never read: the dense operator replaces the kernel product
    dp_.kernel = CIQ_KERNEL_RBF;
    dp_.n_lengthscale = 1;
    dp_.lengthscale = &one;
    dp_.outputscale = 1.0;
    dp_.noise = 0.0;
    const DenseOp dop{thn, M};
    ciq_info si{};
    {
        const void* bp[1] = {a};
        void* op[1] = {c};
        STCHK(solve<double>(1, &dp_, &so, bp, nb, nb, op, nb, nullptr, CIQ_INVSQRT, &si, stream, nullptr, nullptr,
                            &dop));
    }
    if (info_solve) *info_solve = si;
    HIPCHK(launch_svgp_stats(a, c, theta, M, nb, z->outputscale, mean, var, stream));
    if (a_out) HIPCHK(hipMemcpyAsync(a_out, a, (size_t)M * nb * sizeof(double), hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return CIQ_OK;
}

int ciq_svgp_ngd_step(int M, int nb, const double* a, const double* mean, const double* c_mean, const double* c_var,
                      double scale, double step, double* theta, double* Theta, hipStream_t stream) {
    if (M < 1 || nb < 1 || !a || !mean || !c_mean || !c_var || !theta || !Theta) return CIQ_EINVAL;
    if (!std::isfinite(scale) || !std::isfinite(step)) return CIQ_EINVAL;
    int dev;
    STCHK(get_device(&dev));
    ScratchLock lock(dev);
    Sizer sz;
    sz.take<double>((size_t)M * nb);
    sz.take<double>(nb);
    void* base = nullptr;
    STCHK(scratch_reserve(dev, sz.off + 4096, &base));
    Carver c(base);
    double* T = c.take<double>((size_t)M * nb);
    double* u = c.take<double>(nb);
    HIPCHK(launch_ngd_prep(a, mean, c_mean, c_var, M, nb, scale, step, T, u, stream));
    // Theta <- (1 - step) Theta + a T - (step / 2) I;  theta <- (1 - step) theta + a u
    HIPCHK(launch_lr_apply(1.0 - step, Theta, M, a, nb, T, M, M, nb, M, Theta, M, nullptr, nullptr, nullptr, stream));
    HIPCHK(launch_diag_add(Theta, M, -0.5 * step, stream));
    HIPCHK(launch_lr_apply(1.0 - step, theta, 1, a, nb, u, 1, M, nb, 1, theta, 1, nullptr, nullptr, nullptr, stream));
    HIPCHK(hipStreamSynchronize(stream));   // the scratch is reused by the next call
    return CIQ_OK;
}

int ciq_pivoted_cholesky(const ciq_problem* p, int dtype, int rank, double* l_out, int* piv_out,
                         double* trace_out, hipStream_t stream) {
    if (!valid_problem(p) || !valid_dtype(dtype) || !l_out || !piv_out) return CIQ_EINVAL;
    if (rank < 1 || rank > std::min(p->n, CIQ_MAX_RANK)) return CIQ_EINVAL;
    const int n = p->n, dp = p->d;
    double scale[CIQ_MAX_D], ones[CIQ_MAX_D];
    point_scale(p, dtype, scale);
    int ard = 0;
    for (int k = 0; k < CIQ_MAX_D; ++k) {
        ones[k] = 1.0;
        if (k >= p->d) scale[k] = 0.0;
        else if (scale[k] != scale[0]) ard = 1;
    }
    DevAlloc mem;
    PcholScratch w{};
    size_t off = 0;
    double* xh = nullptr;
    auto layout = [&](char* base) {
        off = 0;
        xh = carve<double>(base, off, (size_t)n * dp);
        pchol_layout(n, rank, [&](size_t c) { return carve<double>(base, off, c); }, w);
    };
    layout(nullptr);
    if (!dev_malloc(&mem.p, off, false)) {
        (void)hipGetLastError();
        mem.p = nullptr;
        return CIQ_ENOMEM;
    }
    layout(static_cast<char*>(mem.p));
    hipError_t e;
    if (dtype == CIQ_F64)
        e = launch_prep<double>(static_cast<const double*>(p->x), n, p->d, dp, ones, xh, stream);
    else
        e = launch_prep<float>(static_cast<const float*>(p->x), n, p->d, dp, ones, xh, stream);
    if (e != hipSuccess) return CIQ_EHIP;
    std::vector<int> piv;
    double tr = 0.0;
    STCHK(pchol_run(xh, n, dp, p->kernel, ard, scale, p->outputscale, rank, l_out, rank, w, piv, &tr, stream));
    std::memcpy(piv_out, piv.data(), (size_t)rank * sizeof(int));
    if (trace_out) *trace_out = tr;
    return CIQ_OK;
}

}  // extern "C"
