// Host FP64 quadrature for K^{-1/2} (Appendix B; Alg. S2) and the small
// symmetric eigensolver used by the extreme-eigenvalue estimate.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "ciq.h"

namespace ciq {

// Arithmetic-geometric mean of (1, b), 0 < b <= 1 (Abramowitz & Stegun 17.6).
static double agm1(double b) {
    double a = 1.0;
    for (int it = 0; it < 64; ++it) {
        const double an = 0.5 * (a + b);
        const double bn = std::sqrt(a * b);
        a = an;
        b = bn;
        if (std::fabs(a - b) <= 1e-17 * a) break;
    }
    return 0.5 * (a + b);
}

// Jacobi sn, cn, dn of (u | m) given b0 = sqrt(1 - m) and c0 = sqrt(m), by the
// AGM / descending Landen scale (Abramowitz & Stegun 16.4): a_0 = 1, b_0, c_0;
// a_n = (a + b)/2, b_n = sqrt(a b), c_n = c_{n-1}^2 / (4 a_n); phi_N = 2^N a_N u;
// phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2. dn is taken from
// dn^2 = cn^2 + b0^2 sn^2, which has no cancellation as m -> 1.
static void jacobi_sncndn(double u, double b0, double c0, double* sn, double* cn, double* dn) {
    double a[40], c[40];
    a[0] = 1.0;
    c[0] = c0;
    double b = b0;
    int N = 0;
    while (N < 38) {
        const double an = 0.5 * (a[N] + b);
        const double bn = std::sqrt(a[N] * b);
        const double cn_ = c[N] * c[N] / (4.0 * an);
        ++N;
        a[N] = an;
        c[N] = cn_;
        b = bn;
        if (std::fabs(cn_) <= 1e-18 * an) break;
    }
    double phi = std::ldexp(a[N] * u, N);
    for (int n = N; n >= 1; --n) phi = 0.5 * (phi + std::asin(c[n] * std::sin(phi) / a[n]));
    *sn = std::sin(phi);
    *cn = std::cos(phi);
    *dn = std::sqrt((*cn) * (*cn) + b0 * b0 * (*sn) * (*sn));
}

// Shifts and weights of the HHT rule (positive pair of Appendix B):
//   k^2 = lmin/lmax, K' = K(k') = pi / (2 AGM(1, k)),
//   (sn, cn, dn) = (sn, cn, dn)(u_q K' | k'^2),  u_q = (q - 1/2)/Q,
//   t_q = lmin (sn/cn)^2,  w_q = 2 sqrt(lmin) K' dn / (pi Q cn^2).
// For u_q > 1/2 the quarter-period reflection (A&S 16.8: sn(K - v) = cn v/dn v,
// cn(K - v) = k sn v / dn v, dn(K - v) = k / dn v, with k the complementary
// modulus of k') is used with v = (1 - u_q) K', so the small cn is formed
// without cancellation:
//   t_q = lmax (cn_v / sn_v)^2,   w_q = 2 sqrt(lmax) K' dn_v / (pi Q sn_v^2).
int hht_quadrature(double lmin, double lmax, int Q, double* t, double* w) {
    const double k = std::sqrt(lmin / lmax);                   // modulus k
    const double kp = std::sqrt((1.0 - k) * (1.0 + k));         // complementary k'
    const double Kp = M_PI / (2.0 * agm1(k));                   // K(k') with b0 = sqrt(1 - k'^2) = k
    for (int q = 1; q <= Q; ++q) {
        const double uq = (q - 0.5) / Q;
        double sn, cn, dn;
        if (uq <= 0.5) {
            jacobi_sncndn(uq * Kp, k, kp, &sn, &cn, &dn);
            t[q - 1] = lmin * (sn / cn) * (sn / cn);
            w[q - 1] = 2.0 * std::sqrt(lmin) * Kp * dn / (M_PI * Q * cn * cn);
        } else {
            const double v = ((Q - q + 0.5) / Q) * Kp;
            jacobi_sncndn(v, k, kp, &sn, &cn, &dn);
            t[q - 1] = lmax * (cn / sn) * (cn / sn);
            w[q - 1] = 2.0 * std::sqrt(lmax) * Kp * dn / (M_PI * Q * sn * sn);
        }
    }
    return CIQ_OK;
}

// Eigenvalues/vectors of a small symmetric matrix (row-major n x n) by cyclic
// Jacobi rotations (Golub & Van Loan 8.5). Eigenvector j is column j of v.
// The eigenvectors are accumulated as rows of V^T (contiguous updates).
void sym_eig_jacobi(int n, std::vector<double>& a, std::vector<double>& evals, std::vector<double>& v) {
    std::vector<double> vt((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) vt[(size_t)i * n + i] = 1.0;
    double norm = 0.0;
    for (double x : a) norm += x * x;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += a[(size_t)i * n + j] * a[(size_t)i * n + j];
        if (off <= 1e-30 * norm || off == 0.0) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                double* ap = &a[(size_t)p * n];
                double* aq = &a[(size_t)q * n];
                for (int k = 0; k < n; ++k) {
                    const double apk = ap[k], aqk = aq[k];
                    ap[k] = c * apk - s * aqk;
                    aq[k] = s * apk + c * aqk;
                }
                double* vp = &vt[(size_t)p * n];
                double* vq = &vt[(size_t)q * n];
                for (int k = 0; k < n; ++k) {
                    const double x = vp[k], y = vq[k];
                    vp[k] = c * x - s * y;
                    vq[k] = s * x + c * y;
                }
            }
        }
    }
    evals.resize(n);
    for (int i = 0; i < n; ++i) evals[i] = a[(size_t)i * n + i];
    v.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) v[(size_t)k * n + j] = vt[(size_t)j * n + k];
}

// Fork-join helpers of the eigensolver below: a team of host threads (the
// caller is member 0) that meets at a sense-reversing spin barrier.
namespace {
class SpinBarrier {
  public:
    explicit SpinBarrier(int n) : n_(n) {}
    void wait() {
        const int gen = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
            count_.store(0, std::memory_order_relaxed);
            gen_.store(gen + 1, std::memory_order_release);
        } else {
            while (gen_.load(std::memory_order_acquire) == gen) std::this_thread::yield();
        }
    }

  private:
    const int n_;
    std::atomic<int> count_{0};
    std::atomic<int> gen_{0};
};

// Threads for an n x n problem: at most 16 (and the machine's count), one
// per 48 rows, one below n = 128.
int team_size(int n) {
    if (n < 128) return 1;
    const unsigned hw = std::thread::hardware_concurrency();
    const int cap = (int)std::min(hw == 0 ? 1u : hw, 16u);
    return std::max(1, std::min(cap, n / 48));
}

template <typename F>
void run_team(int T, F&& f) {
    std::vector<std::thread> th;
    th.reserve(T > 1 ? T - 1 : 0);
    for (int t = 1; t < T; ++t) th.emplace_back([&f, t] { f(t); });
    f(0);
    for (auto& x : th) x.join();
}

struct Givens {
    int k;
    double c, s;
};
}  // namespace

// Eigenvalues/vectors of a symmetric matrix (row-major n x n, overwritten) for
// the larger matrices of the preconditioner: Householder reduction to
// tridiagonal form, then implicit symmetric QR steps with the Wilkinson shift
// and deflation (Golub & Van Loan 8.3.1, 8.3.3), ~9 n^3 flops against the
// ~30 n^3 of cyclic Jacobi. The orthogonal factor V^T = G_last ... G_1
// H_{n-3} ... H_0 is formed after both phases from the stored reflectors and
// the recorded rotations: every factor acts on the columns of V^T one by one,
// so a team of threads takes one slice of columns each. The reduction itself
// splits its matrix-vector product and rank-2 update by rows. Each element
// sees the same operations in the same order for any team size, so the
// result does not depend on the thread count. Eigenvector j is column j of v.
void sym_eig_tridiag(int n, std::vector<double>& a, std::vector<double>& evals, std::vector<double>& v) {
    const int T = team_size(n);
    std::vector<double> hvs((size_t)n * n, 0.0);   // reflector k in row k, entries k+1..n-1
    std::vector<double> betas(n, 0.0);             // 0: no reflector at step k
    std::vector<double> p(n);
    SpinBarrier bar(T);
    // ---- Householder reduction: A <- H_k A H_k on the trailing block
    run_team(T, [&](int t) {
        std::vector<double> hv(n), w(n);
        for (int k = 0; k + 2 < n; ++k) {
            const int m = n - k - 1;
            const double* x = &a[(size_t)k * n + k + 1];
            double sig = 0.0;
            for (int i = 0; i < m; ++i) sig += x[i] * x[i];
            sig = std::sqrt(sig);
            if (sig == 0.0) continue;                    // the same on every member
            const double alpha = (x[0] >= 0.0) ? -sig : sig;
            for (int i = 0; i < m; ++i) hv[i] = x[i];
            hv[0] -= alpha;
            double vv = 0.0;
            for (int i = 0; i < m; ++i) vv += hv[i] * hv[i];
            const double beta = 2.0 / vv;
            const int i0 = (int)((long long)m * t / T), i1 = (int)((long long)m * (t + 1) / T);
            for (int i = i0; i < i1; ++i) {
                const double* ai = &a[(size_t)(k + 1 + i) * n + k + 1];
                double s = 0.0;
                for (int j = 0; j < m; ++j) s += ai[j] * hv[j];
                p[i] = beta * s;
            }
            bar.wait();                                  // p complete
            double vp = 0.0;
            for (int i = 0; i < m; ++i) vp += hv[i] * p[i];
            const double kc = 0.5 * beta * vp;
            for (int i = 0; i < m; ++i) w[i] = p[i] - kc * hv[i];
            bar.wait();                                  // p read by all before rows change
            for (int i = i0; i < i1; ++i) {
                double* ai = &a[(size_t)(k + 1 + i) * n + k + 1];
                const double vi = hv[i], wi = w[i];
                for (int j = 0; j < m; ++j) ai[j] -= vi * w[j] + wi * hv[j];
            }
            if (t == 0) {
                betas[k] = beta;
                for (int i = 0; i < m; ++i) hvs[(size_t)k * n + k + 1 + i] = hv[i];
                a[(size_t)k * n + k + 1] = alpha;
                for (int j = k + 2; j < n; ++j) a[(size_t)k * n + j] = 0.0;
            }
            bar.wait();                                  // rows updated before the next reflector
        }
    });
    std::vector<double> d(n), e(n > 1 ? n - 1 : 1, 0.0);
    for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = a[(size_t)i * n + i + 1];
    // ---- implicit symmetric QR on (d, e) with deflation; rotations recorded
    std::vector<Givens> rot;
    const double eps = 2.220446049250313e-16;
    auto negligible = [&](int i) { return std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1])); };
    int hi = n - 1, guard = 0;
    while (hi > 0 && guard < 64 * n) {
        if (negligible(hi - 1)) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !negligible(lo - 1)) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        ++guard;
        // Wilkinson shift from the trailing 2 x 2 of the block [lo, hi]
        const double dl = 0.5 * (d[hi - 1] - d[hi]);
        const double b2 = e[hi - 1] * e[hi - 1];
        const double mu = d[hi] - b2 / (dl + ((dl >= 0.0) ? 1.0 : -1.0) * std::sqrt(dl * dl + b2));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            // Givens (c, s): c x - s z = r, s x + c z = 0
            double c = 1.0, s = 0.0;
            if (z != 0.0) {
                if (std::fabs(z) > std::fabs(x)) {
                    const double tau = -x / z;
                    s = 1.0 / std::sqrt(1.0 + tau * tau);
                    c = s * tau;
                } else {
                    const double tau = -z / x;
                    c = 1.0 / std::sqrt(1.0 + tau * tau);
                    s = c * tau;
                }
            }
            if (k > lo) e[k - 1] = c * x - s * z;   // bulge chased out of column k - 1
            const double ak = d[k], bk = e[k], ck = d[k + 1];
            d[k] = c * c * ak - 2.0 * c * s * bk + s * s * ck;
            d[k + 1] = s * s * ak + 2.0 * c * s * bk + c * c * ck;
            e[k] = c * s * (ak - ck) + (c * c - s * s) * bk;
            if (k + 1 < hi) {
                z = -s * e[k + 1];               // new bulge at (k + 2, k)
                e[k + 1] = c * e[k + 1];
                x = e[k];
            }
            rot.push_back(Givens{k, c, s});
        }
    }
    // ---- V^T, one slice of columns per member in a compact local copy
    // (row i of the slice at i * width); member t then writes rows j0..j1 of
    // v, which are the slice's columns
    v.assign((size_t)n * n, 0.0);
    run_team(T, [&](int t) {
        const int j0 = (int)((long long)n * t / T), j1 = (int)((long long)n * (t + 1) / T);
        const int wdt = j1 - j0;
        if (wdt <= 0) return;
        std::vector<double> sl((size_t)n * wdt, 0.0), u(wdt);
        for (int j = j0; j < j1; ++j) sl[(size_t)j * wdt + (j - j0)] = 1.0;
        for (int k = 0; k + 2 < n; ++k) {
            if (betas[k] == 0.0) continue;
            const int m = n - k - 1;
            const double* hv = &hvs[(size_t)k * n + k + 1];
            for (int j = 0; j < wdt; ++j) u[j] = 0.0;
            for (int i = 0; i < m; ++i) {
                const double* ri = &sl[(size_t)(k + 1 + i) * wdt];
                const double vi = hv[i];
                for (int j = 0; j < wdt; ++j) u[j] += vi * ri[j];
            }
            for (int i = 0; i < m; ++i) {
                double* ri = &sl[(size_t)(k + 1 + i) * wdt];
                const double f = betas[k] * hv[i];
                for (int j = 0; j < wdt; ++j) ri[j] -= f * u[j];
            }
        }
        for (const Givens& g : rot) {
            double* rk = &sl[(size_t)g.k * wdt];
            double* rk1 = &sl[(size_t)(g.k + 1) * wdt];
            for (int j = 0; j < wdt; ++j) {
                const double y0 = rk[j], y1 = rk1[j];
                rk[j] = g.c * y0 - g.s * y1;
                rk1[j] = g.s * y0 + g.c * y1;
            }
        }
        for (int k = j0; k < j1; ++k)
            for (int j = 0; j < n; ++j) v[(size_t)k * n + j] = sl[(size_t)j * wdt + (k - j0)];
    });
    evals = d;
}

// Widened bounds from a Lanczos tridiagonal (alpha[0..J), beta[0..J), beta[J-1]
// the final residual norm): lambda_max = theta_max + beta_{J+1} |y_J|,
// lambda_min = min(theta_min, noise) if noise > 0, else theta_min / 2.
void bounds_from_tridiag(int J, const double* alpha, const double* beta, double noise, double* lmin,
                         double* lmax) {
    std::vector<double> a((size_t)J * J, 0.0), ev, v;
    for (int i = 0; i < J; ++i) {
        a[(size_t)i * J + i] = alpha[i];
        if (i + 1 < J) a[(size_t)i * J + i + 1] = a[(size_t)(i + 1) * J + i] = beta[i];
    }
    sym_eig_jacobi(J, a, ev, v);
    int imin = 0, imax = 0;
    for (int i = 1; i < J; ++i) {
        if (ev[i] < ev[imin]) imin = i;
        if (ev[i] > ev[imax]) imax = i;
    }
    const double ylast = v[(size_t)(J - 1) * J + imax];
    *lmax = ev[imax] + std::fabs(beta[J - 1] * ylast);
    *lmin = (noise > 0.0) ? std::fmin(ev[imin], noise) : 0.5 * ev[imin];
}

}  // namespace ciq
