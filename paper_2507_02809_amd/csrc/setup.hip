// Host-side set-up of a problem: validation, the stencil a_l of the discrete fractional
// Laplacian (§4 eqs. fourier-coeff and fourier-coeff-1d), the eigenvalues of its circulant
// embedding (§5 matvec step 1(b)), the tau eigenvalues (§5 Remark), the L1 weights
// (§4 eq. L1-formula and the e_m definition), and the device copies.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <thread>

#include "internal.hpp"

namespace tsfde {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

const char* last_error() { return g_err; }

// parallel for over [0, n) on the host
template <typename F>
static void parallel_for(long long n, F&& f) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 64 || nt == 1) {
        for (long long i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (long long i = t; i < n; i += nt) f(i);
        });
    for (auto& x : th) x.join();
}

// cos(2 pi m / K) table, m = 0..K-1
static std::vector<double> cos_table(long long K) {
    std::vector<double> c(K);
    for (long long m = 0; m < K; ++m) c[m] = std::cos(2.0 * M_PI * (double)m / (double)K);
    return c;
}

// ---- stencil -------------------------------------------------------------

// d = 1: a_0 = Gamma(omega+1)/Gamma(omega/2+1)^2, a_{l+1} = (1 - (omega+1)/(omega/2+l+1)) a_l (Lemma 1)
static void stencil_1d(int N, double omega, double* a) {
    a[0] = std::tgamma(omega + 1.0) / std::pow(std::tgamma(omega / 2.0 + 1.0), 2);
    for (int l = 0; l + 1 < N; ++l) a[l + 1] = (1.0 - (omega + 1.0) / (omega / 2.0 + l + 1.0)) * a[l];
}

// in-place iterative radix-2 FFT (exp(-2 pi i jk/K)), host side, K a power of two
static void host_fft(std::vector<std::complex<double>>& x, const std::vector<std::complex<double>>& w) {
    const size_t K = x.size();
    for (size_t i = 1, j = 0; i < K; ++i) {
        size_t bit = K >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    for (size_t len = 2; len <= K; len <<= 1) {
        const size_t step = K / len;
        for (size_t i = 0; i < K; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> u = x[i + k], v = x[i + k + len / 2] * w[k * step];
                x[i + k] = u + v;
                x[i + k + len / 2] = u - v;
            }
    }
}

// d = 2, grid size K: a^K_l = K^-2 sum_k g(2 pi k/K) cos(2 pi k.l/K), the trapezoidal rule for
// eq. fourier-coeff.  Rows k1 in [0, K/2] (g is even in each variable) are transformed over k2 with
// the FFT, then the k1 sum is done directly with weights 1, 2, .., 2, 1.
static void stencil_2d_grid(int N, double omega, long long K, std::vector<double>& a) {
    const long long Kh = K / 2;
    std::vector<double> s(K), w(Kh + 1);
    for (long long k = 0; k < K; ++k) {
        const double sn = std::sin(M_PI * (double)k / (double)K);
        s[k] = 4.0 * sn * sn;
    }
    for (long long k = 0; k <= Kh; ++k) w[k] = (k == 0 || k == Kh) ? 1.0 : 2.0;
    std::vector<std::complex<double>> tw(K / 2);
    for (long long k = 0; k < K / 2; ++k) tw[k] = std::polar(1.0, -2.0 * M_PI * (double)k / (double)K);
    // stage 1: G[k1][l2] = sum_{k2=0}^{K-1} g(k1,k2) cos(2 pi k2 l2 / K); two rows per complex FFT
    std::vector<double> G((Kh + 1) * (size_t)N);
    const long long npair = (Kh + 2) / 2;
    parallel_for(npair, [&](long long pr) {
        const long long k1a = 2 * pr, k1b = 2 * pr + 1;
        std::vector<std::complex<double>> x(K);
        for (long long k2 = 0; k2 < K; ++k2) {
            const double ga = std::pow(s[k1a] + s[k2], omega / 2.0);
            const double gb = (k1b <= Kh) ? std::pow(s[k1b] + s[k2], omega / 2.0) : 0.0;
            x[k2] = {ga, gb};
        }
        host_fft(x, tw);
        // rows are real and even: their transforms are real; packed as X = A + i B
        for (int l2 = 0; l2 < N; ++l2) {
            G[k1a * N + l2] = x[l2].real();
            if (k1b <= Kh) G[k1b * N + l2] = x[l2].imag();
        }
    });
    std::vector<double> ct(K);
    for (long long m = 0; m < K; ++m) ct[m] = std::cos(2.0 * M_PI * (double)m / (double)K);
    // stage 2: a[l1][l2] = K^-2 sum_k1 w cos(2 pi k1 l1/K) G[k1][l2]
    a.assign((size_t)N * N, 0.0);
    const double inv = 1.0 / ((double)K * (double)K);
    parallel_for(N, [&](long long l1) {
        for (int l2 = 0; l2 < N; ++l2) {
            double acc = 0.0;
            long long idx = 0;
            for (long long k1 = 0; k1 <= Kh; ++k1) {
                acc += w[k1] * ct[idx] * G[k1 * N + l2];
                idx += l1;
                if (idx >= K) idx -= K;
            }
            a[l1 * N + l2] = acc * inv;
        }
    });
}

// d = 2: trapezoidal grids K/4, K/2 and K with K >= 64 N, Richardson-extrapolated twice.  The
// generating function vanishes like |theta|^omega at the origin, so the trapezoidal error expands in
// K^-(2+omega), K^-(4+omega), ...; two extrapolation steps leave O(K^-(6+omega)).
static void stencil_2d(int N, double omega, double* out) {
    long long K = 1024;
    while (K < 64LL * N) K *= 2;
    std::vector<double> a4, a2, a1;
    stencil_2d_grid(N, omega, K / 4, a4);
    stencil_2d_grid(N, omega, K / 2, a2);
    stencil_2d_grid(N, omega, K, a1);
    const double r0 = std::pow(2.0, 2.0 + omega), r1 = std::pow(2.0, 4.0 + omega);
    for (size_t i = 0; i < a1.size(); ++i) {
        const double e1 = (r0 * a2[i] - a4[i]) / (r0 - 1.0);
        const double e2 = (r0 * a1[i] - a2[i]) / (r0 - 1.0);
        out[i] = (r1 * e2 - e1) / (r1 - 1.0);
    }
}

// ---- spectra ---------------------------------------------------------------

// eigenvalues of the circulant embedding (size L per direction) divided by L^d;
// d = 1: sym[k]; d = 2: sym[k2 * L + k1] for k2 < L/2+1
static std::vector<double> circulant_symbol(int d, int N, int L, const std::vector<double>& a) {
    const std::vector<double> ct = cos_table(L);
    const int H = L / 2 + 1;
    if (d == 1) {
        std::vector<double> sym(L);
        for (int k = 0; k < L; ++k) {
            double acc = a[0];
            long long idx = 0;
            for (int l = 1; l < N; ++l) {
                idx += k;
                idx %= L;
                acc += 2.0 * a[l] * ct[idx];
            }
            sym[k] = acc / L;
        }
        return sym;
    }
    std::vector<double> G((size_t)N * H);  // G[l1][k2]
    parallel_for(N, [&](long long l1) {
        for (int k2 = 0; k2 < H; ++k2) {
            double acc = 0.0;
            long long idx = 0;
            for (int l2 = 0; l2 < N; ++l2) {
                acc += (l2 == 0 ? 1.0 : 2.0) * a[l1 * N + l2] * ct[idx];
                idx += k2;
                if (idx >= L) idx -= L;
            }
            G[l1 * H + k2] = acc;
        }
    });
    std::vector<double> sym((size_t)H * L);
    const double inv = 1.0 / ((double)L * (double)L);
    parallel_for(H, [&](long long k2) {
        for (int k1 = 0; k1 < L; ++k1) {
            double acc = 0.0;
            long long idx = 0;
            for (int l1 = 0; l1 < N; ++l1) {
                acc += (l1 == 0 ? 1.0 : 2.0) * ct[idx] * G[(size_t)l1 * H + k2];
                idx += k1;
                if (idx >= L) idx -= L;
            }
            sym[k2 * L + k1] = acc * inv;
        }
    });
    return sym;
}

// natural tau eigenvalues: sum_{|l_i|<N} a_|l| prod cos(l_i theta_{k_i}), theta_k = k pi/(N+1), k = 1..N
static std::vector<double> tau_eigs(int d, int N, const std::vector<double>& a) {
    const long long P2 = 2LL * (N + 1);
    const std::vector<double> ct = cos_table(P2);  // cos(pi m/(N+1))
    auto cosk = [&](long long l, long long k) { return ct[(l * k) % P2]; };
    if (d == 1) {
        std::vector<double> t(N);
        for (int k = 0; k < N; ++k) {
            double acc = a[0];
            for (int l = 1; l < N; ++l) acc += 2.0 * a[l] * cosk(l, k + 1);
            t[k] = acc;
        }
        return t;
    }
    std::vector<double> G((size_t)N * N);  // G[l1][k2]
    parallel_for(N, [&](long long l1) {
        for (int k2 = 0; k2 < N; ++k2) {
            double acc = 0.0;
            for (int l2 = 0; l2 < N; ++l2) acc += (l2 == 0 ? 1.0 : 2.0) * a[l1 * N + l2] * cosk(l2, k2 + 1);
            G[l1 * N + k2] = acc;
        }
    });
    std::vector<double> t((size_t)N * N);
    parallel_for(N, [&](long long k1) {
        for (int k2 = 0; k2 < N; ++k2) {
            double acc = 0.0;
            for (int l1 = 0; l1 < N; ++l1) acc += (l1 == 0 ? 1.0 : 2.0) * cosk(l1, k1 + 1) * G[(size_t)l1 * N + k2];
            t[(size_t)k2 * N + k1] = acc;  // stored [k2][k1]: row k2 holds the k1 values
        }
    });
    return t;
}

// T_{n,S} blocks solved by dense sine transforms (any N): tab[m] = sin(pi m/(N+1)), m < 2(N+1), and the
// tau eigenvalues of B_N as lam[k1][k2] (k2 the frequency of the fast index; 1D: lam[k]); returns the
// smallest eigenvalue.
double tau_dense_tables(const Problem& P, std::vector<double>& tab, std::vector<double>& lam) {
    const int N = P.N;
    const long long P2 = 2LL * (N + 1);
    tab.resize(P2);
    for (long long m = 0; m < P2; ++m) tab[m] = std::sin(M_PI * (double)m / (double)(N + 1));
    const std::vector<double> t = tau_eigs(P.d, N, P.stencil);
    if (P.d == 1) {
        lam = t;
    } else {
        lam.resize((size_t)N * N);
        for (int k1 = 0; k1 < N; ++k1)
            for (int k2 = 0; k2 < N; ++k2) lam[(size_t)k1 * N + k2] = t[(size_t)k2 * N + k1];
    }
    return *std::min_element(lam.begin(), lam.end());
}

// Strang's circulant s(B) (§5.1 Remark): first column c_l = a_{f(l)} per level with f(l) = l for
// l <= N/2 and N - l above (the central diagonals wrapped around).  cas[m] = cos + sin of 2 pi m/N,
// lam[k1][k2] = sum_l c[l1][l2] cos(2 pi l1 k1/N) cos(2 pi l2 k2/N), its eigenvalues in the Hartley
// basis (1D: lam[k]); returns the smallest eigenvalue.  The sums cancel heavily at the smallest
// eigenvalues (the stencil's entries nearly sum to zero), so they are accumulated in long double.
double strang_tables(const Problem& P, std::vector<double>& cas, std::vector<double>& lam) {
    const int N = P.N;
    std::vector<long double> ct(N);
    for (int m = 0; m < N; ++m) ct[m] = std::cos(2.0L * (long double)M_PI * (long double)m / (long double)N);
    cas.resize(N);
    for (int m = 0; m < N; ++m) cas[m] = std::cos(2.0 * M_PI * m / N) + std::sin(2.0 * M_PI * m / N);
    auto f = [N](int l) { return l <= N / 2 ? l : N - l; };
    auto cosk = [&](long long l, long long k) { return ct[(l * k) % N]; };
    const std::vector<double>& a = P.stencil;
    if (P.d == 1) {
        lam.assign(N, 0.0);
        for (int k = 0; k < N; ++k) {
            long double acc = 0.0L;
            for (int l = 0; l < N; ++l) acc += (long double)a[f(l)] * cosk(l, k);
            lam[k] = (double)acc;
        }
    } else {
        std::vector<long double> G((size_t)N * N);  // G[l1][k2]
        parallel_for(N, [&](long long l1) {
            const double* row = a.data() + (size_t)f((int)l1) * N;
            for (int k2 = 0; k2 < N; ++k2) {
                long double acc = 0.0L;
                for (int l2 = 0; l2 < N; ++l2) acc += (long double)row[f(l2)] * cosk(l2, k2);
                G[(size_t)l1 * N + k2] = acc;
            }
        });
        lam.assign((size_t)N * N, 0.0);
        parallel_for(N, [&](long long k1) {
            for (int k2 = 0; k2 < N; ++k2) {
                long double acc = 0.0L;
                for (int l1 = 0; l1 < N; ++l1) acc += cosk(l1, k1) * G[(size_t)l1 * N + k2];
                lam[(size_t)k1 * N + k2] = (double)acc;
            }
        });
    }
    return *std::min_element(lam.begin(), lam.end());
}

static std::vector<double> twiddles(int L) {
    std::vector<double> t(2 * (size_t)L);
    for (int m = 0; m < L; ++m) {
        const double ang = 2.0 * M_PI * (double)m / (double)L;
        t[2 * m] = std::cos(ang);
        t[2 * m + 1] = -std::sin(ang);
    }
    return t;
}

// ---- device upload -----------------------------------------------------------

template <typename T>
static T* upload(Problem& P, const double* src, size_t n) {
    T* d = nullptr;
    TSFDE_HIP(hipMalloc(&d, sizeof(T) * std::max<size_t>(n, 1)));
    P.bytes += sizeof(T) * n;
    if (n) {
        std::vector<T> tmp(src, src + n);
        TSFDE_HIP(hipMemcpy(d, tmp.data(), sizeof(T) * n, hipMemcpyHostToDevice));
    }
    return d;
}

template <typename T>
static T* alloc(Problem& P, size_t n) {
    T* d = nullptr;
    TSFDE_HIP(hipMalloc(&d, sizeof(T) * std::max<size_t>(n, 1)));
    P.bytes += sizeof(T) * n;
    return d;
}

template <typename T>
static void build_dev(Problem& P, Dev<T>& D, const std::vector<double>& dg, const std::vector<double>& epad,
                      const std::vector<double>& sym, const std::vector<double>& tw, const std::vector<double>& twd,
                      const std::vector<double>& tau) {
    const size_t MN = (size_t)P.M * P.Nd;
    D.gamma1 = upload<T>(P, P.gamma1_h.data(), MN);
    D.gamma2 = upload<T>(P, P.gamma2_h.data(), MN);
    D.dg = upload<T>(P, dg.data(), MN);
    D.epad = upload<T>(P, epad.data(), epad.size());
    D.q = upload<T>(P, P.q_h.data(), P.M);
    D.sym = upload<T>(P, sym.data(), sym.size());
    D.tw = reinterpret_cast<cplx<T>*>(upload<T>(P, tw.data(), tw.size()));
    if (!twd.empty()) D.twd = reinterpret_cast<cplx<T>*>(upload<T>(P, twd.data(), twd.size()));
    if (!tau.empty()) D.tau = upload<T>(P, tau.data(), tau.size());
    // row stride of the matvec spectra: N rounded up to 16 (the other users take stride N)
    if (P.d == 2) D.spec = reinterpret_cast<cplx<T>*>(alloc<T>(P, 2 * (size_t)P.nspec * P.H * (size_t)((P.N + 15) & ~15)));
    D.pcg = alloc<T>(P, 8 * (size_t)P.Nd);
    D.partial = alloc<T>(P, kMaxPartials);
}

template <typename T>
static void free_dev(Dev<T>& D) {
    void* ptrs[] = {D.gamma1, D.gamma2, D.dg, D.epad, D.q, D.sym, D.tw, D.twd, D.tau, D.spec, D.pcg, D.partial,
                    D.vecA, D.vecB};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    D = Dev<T>{};
}

void free_problem(Problem* P) {
    if (!P) return;
    free_dev(P->f64);
    free_dev(P->f32);
    pinv_persistent_free<double>(P->pw64);
    pinv_persistent_free<float>(P->pw32);
    void* ptrs[] = {P->d_bw, P->d_rho, P->d_mu, P->z_rhs, P->xbuf, P->V, P->Z, P->arn_part, P->arn_h, P->rwork, P->adj_u,
                    P->dev_scalars, P->strang64, P->strang32, P->strang_hist, P->refine_work, P->vjp_work,
                    P->d_sigma, P->fwd_work, P->taud64, P->taud32, P->spec_work, P->dense_bar, P->blk_V, P->blk_part,
                    P->blk_small, P->blk_io, P->adj_rev};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (P->host_scalars) (void)hipHostFree(P->host_scalars);
    if (P->multi_dev) (void)hipFree(P->multi_dev);
    if (P->multi_host) (void)hipHostFree(P->multi_host);
    if (P->cyc_exec) (void)hipGraphExecDestroy(P->cyc_exec);
    if (P->cyc_stream) (void)hipStreamDestroy(P->cyc_stream);
    if (P->cyc_h) (void)hipFree(P->cyc_h);
    if (P->cyc_h_host) (void)hipHostFree(P->cyc_h_host);
    if (P->mv_fork) (void)hipEventDestroy(P->mv_fork);
    if (P->mv_join) (void)hipEventDestroy(P->mv_join);
    if (P->mv_aux) (void)hipStreamDestroy(P->mv_aux);
    delete P;
}

static bool finite_all(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

tsfde_status compute_stencil(int d, int N, double omega, double* out) {
    if ((d != 1 && d != 2) || N < 1 || !(omega > 1.0 && omega < 2.0) || !out) {
        set_error("compute_stencil: need d in {1,2}, N >= 1, 1 < omega < 2, out != NULL");
        return TSFDE_EINVAL;
    }
    if (d == 1) stencil_1d(N, omega, out);
    else stencil_2d(N, omega, out);
    return TSFDE_OK;
}

tsfde_status create(int d, int N, int M, double T, double beta, double omega, double alpha, const double* gamma1,
                    const double* gamma2, const double* q, const double* rho, const double* mu, double length,
                    const double* stencil, Problem** out) {
    if (!out) {
        set_error("create_problem: out is NULL");
        return TSFDE_EINVAL;
    }
    *out = nullptr;
    if (d != 1 && d != 2) { set_error("create_problem: d must be 1 or 2 (got %d)", d); return TSFDE_EINVAL; }
    if (N < 1 || M < 1) { set_error("create_problem: need N >= 1 and M >= 1"); return TSFDE_EINVAL; }
    if (!(T > 0.0) || !std::isfinite(T)) { set_error("create_problem: need T > 0"); return TSFDE_EINVAL; }
    if (!(beta > 0.0 && beta < 1.0)) { set_error("create_problem: need 0 < beta < 1"); return TSFDE_EINVAL; }
    if (!(omega > 1.0 && omega < 2.0)) { set_error("create_problem: need 1 < omega < 2"); return TSFDE_EINVAL; }
    if (!(alpha > 0.0) || !std::isfinite(alpha)) { set_error("create_problem: need alpha > 0"); return TSFDE_EINVAL; }
    if (!(length > 0.0) || !std::isfinite(length)) { set_error("create_problem: need length > 0"); return TSFDE_EINVAL; }
    if (!gamma1 || !gamma2 || !q) { set_error("create_problem: gamma1, gamma2 and q are required"); return TSFDE_EINVAL; }
    int L = 8;
    while (L < 2 * N - 1) L *= 2;
    if (L > 8192) {
        set_error("create_problem: N = %d needs a circulant embedding of %d > 8192 points per direction", N, L);
        return TSFDE_EINVAL;
    }
    long long Nd = (d == 1) ? N : (long long)N * N;
    const size_t MN = (size_t)M * Nd;
    if (!finite_all(gamma1, MN) || !finite_all(gamma2, MN) || !finite_all(q, M) || (rho && !finite_all(rho, Nd)) ||
        (mu && !finite_all(mu, Nd)) || (stencil && !finite_all(stencil, Nd))) {
        set_error("create_problem: non-finite value in an input array");
        return TSFDE_ENONFINITE;
    }
    for (size_t i = 0; i < MN; ++i) {
        if (gamma2[i] <= 0.0 || gamma1[i] < 0.0) {
            set_error("create_problem: need gamma1 >= 0 and gamma2 > 0 (index %zu)", i);
            return TSFDE_EINVAL;
        }
    }
    for (int s = 0; s < M; ++s)
        if (q[s] <= 0.0) { set_error("create_problem: need q > 0"); return TSFDE_EINVAL; }

    Problem* P = new Problem();
    try {
        P->d = d; P->N = N; P->M = M; P->T = T; P->beta = beta; P->omega = omega; P->alpha = alpha;
        P->length = length;
        P->Nd = Nd;
        P->ntot = (long long)(M + 1) * Nd;
        P->h = length / (N + 1);
        P->dt = T / M;
        P->eta = std::pow(P->dt, beta) * std::tgamma(2.0 - beta);
        P->ct = P->eta / std::pow(P->h, omega);
        P->cf = alpha / std::pow(P->h, omega);
        // the sine transforms run as FFTs of at least 8 points (the shortest transform the kernels take)
        P->Ld = is_pow2(2LL * (N + 1)) && 2 * (N + 1) >= 8 && 2 * (N + 1) <= 8192 ? 2 * (N + 1) : 0;
        P->tau_ok = P->Ld > 0;
        P->Nt = N;
        if (!P->tau_ok) {
            int Ld = 8;
            while (Ld < 2 * (N + 1)) Ld *= 2;
            if (Ld <= 8192) {
                P->tau_pad = true;
                P->Nt = Ld / 2 - 1;
                P->Ld = Ld;
                L = std::max(L, Ld);  // one transform length serves the Toeplitz product and the sine transform
            }
        }
        P->L = L;
        P->H = L / 2 + 1;
        P->gamma1_h.assign(gamma1, gamma1 + MN);
        P->gamma2_h.assign(gamma2, gamma2 + MN);
        P->q_h.assign(q, q + M);
        P->rho_h.assign(Nd, 0.0);
        if (rho) P->rho_h.assign(rho, rho + Nd);
        P->mu_h.assign(Nd, 0.0);
        if (mu) P->mu_h.assign(mu, mu + Nd);
        // L1 weights (§4): b_m = (m+1)^(1-beta) - m^(1-beta);  e_0 = 1, e_m = b_m - b_{m-1}
        P->b.resize(M);
        P->e.resize(M);
        for (int m = 0; m < M; ++m) P->b[m] = std::pow(m + 1.0, 1.0 - beta) - std::pow((double)m, 1.0 - beta);
        P->e[0] = 1.0;
        for (int m = 1; m < M; ++m)
            P->e[m] = std::pow(m + 1.0, 1.0 - beta) - 2.0 * std::pow((double)m, 1.0 - beta) +
                      std::pow(m - 1.0, 1.0 - beta);
        // stencil
        P->stencil.resize(Nd);
        if (stencil) std::memcpy(P->stencil.data(), stencil, sizeof(double) * Nd);
        else if (d == 1) stencil_1d(N, omega, P->stencil.data());
        else stencil_2d(N, omega, P->stencil.data());
        P->a0 = P->stencil[0];
        // symmetrised diagonal e_0 gamma1/gamma2 and its mean per step (tau preconditioner shift)
        std::vector<double> dg(MN);
        P->sigma.assign(M, 0.0);
        for (int s = 0; s < M; ++s) {
            double acc = 0.0;
            for (long long j = 0; j < Nd; ++j) {
                const size_t o = (size_t)s * Nd + j;
                dg[o] = P->e[0] * gamma1[o] / gamma2[o];
                acc += dg[o];
            }
            P->sigma[s] = acc / Nd;
        }
        std::vector<double> epad(kEpad + M + 64, 0.0);
        for (int m = 0; m < M; ++m) epad[kEpad + m] = P->e[m];
        const std::vector<double> sym = circulant_symbol(d, N, L, P->stencil);
        const std::vector<double> tw = twiddles(L);
        std::vector<double> twd, tau;
        if (P->tau_ok) {
            twd = twiddles(P->Ld);
            tau = tau_eigs(d, N, P->stencil);
        } else if (P->tau_pad) {
            // the stencil continued to Nt entries per direction (the problem's own entries first)
            const int Nt = P->Nt;
            if (d == 1) {
                std::vector<double> ext(Nt);
                stencil_1d(Nt, omega, ext.data());
                std::copy(P->stencil.begin(), P->stencil.end(), ext.begin());
                tau = tau_eigs(1, Nt, ext);
            } else {
                std::vector<double> ext((size_t)Nt * Nt);
                stencil_2d(Nt, omega, ext.data());
                for (int l1 = 0; l1 < N; ++l1)
                    std::copy(P->stencil.begin() + (size_t)l1 * N, P->stencil.begin() + (size_t)(l1 + 1) * N,
                              ext.begin() + (size_t)l1 * Nt);
                tau = tau_eigs(2, Nt, ext);
            }
        }
        P->nspec = (d == 2) ? M + 1 : 0;
        build_dev<double>(*P, P->f64, dg, epad, sym, tw, twd, tau);
        build_dev<float>(*P, P->f32, dg, epad, sym, tw, twd, tau);
        P->have_f32 = true;
        P->d_bw = upload<double>(*P, P->b.data(), M);
        P->d_sigma = upload<double>(*P, P->sigma.data(), M);
        P->d_rho = upload<double>(*P, P->rho_h.data(), Nd);
        P->d_mu = upload<double>(*P, P->mu_h.data(), Nd);
        P->z_rhs = alloc<double>(*P, P->ntot);
        P->dev_scalars = alloc<double>(*P, 64);
        TSFDE_HIP(hipHostMalloc(&P->host_scalars, 64 * sizeof(double), hipHostMallocDefault));
    } catch (const HipError& e) {
        set_error("create_problem: %s failed: %s", e.where.c_str(), hipGetErrorString(e.code));
        const bool oom = (e.code == hipErrorOutOfMemory);
        free_problem(P);
        return oom ? TSFDE_ENOMEM : TSFDE_EDEVICE;
    } catch (const std::bad_alloc&) {
        set_error("create_problem: host allocation failed");
        free_problem(P);
        return TSFDE_ENOMEM;
    }
    *out = P;
    return TSFDE_OK;
}

// copy host values into an existing device array of T
template <typename T>
static void refresh(T* d, const double* src, size_t n) {
    std::vector<T> tmp(src, src + n);
    TSFDE_HIP(hipMemcpy(d, tmp.data(), sizeof(T) * n, hipMemcpyHostToDevice));
}

tsfde_status set_gamma2(Problem* P, const double* gamma2) {
    if (!P || !gamma2) { set_error("set_gamma2: NULL argument"); return TSFDE_EINVAL; }
    const size_t MN = (size_t)P->M * P->Nd;
    if (!finite_all(gamma2, MN)) { set_error("set_gamma2: non-finite value in gamma2"); return TSFDE_ENONFINITE; }
    for (size_t i = 0; i < MN; ++i)
        if (gamma2[i] <= 0.0) { set_error("set_gamma2: need gamma2 > 0 (index %zu)", i); return TSFDE_EINVAL; }
    try {
        P->gamma2_h.assign(gamma2, gamma2 + MN);
        // the symmetrised diagonal e_0 gamma1/gamma2 of every block and its slice means
        std::vector<double> dg(MN);
        for (int s = 0; s < P->M; ++s) {
            double acc = 0.0;
            for (long long j = 0; j < P->Nd; ++j) {
                const size_t o = (size_t)s * P->Nd + j;
                dg[o] = P->e[0] * P->gamma1_h[o] / gamma2[o];
                acc += dg[o];
            }
            P->sigma[s] = acc / P->Nd;
        }
        refresh(P->f64.gamma2, gamma2, MN);
        refresh(P->f64.dg, dg.data(), MN);
        refresh(P->f32.gamma2, gamma2, MN);
        refresh(P->f32.dg, dg.data(), MN);
        TSFDE_HIP(hipMemcpy(P->d_sigma, P->sigma.data(), sizeof(double) * P->M, hipMemcpyHostToDevice));
    } catch (const HipError& e) {
        set_error("set_gamma2: %s failed: %s", e.where.c_str(), hipGetErrorString(e.code));
        return TSFDE_EDEVICE;
    }
    return TSFDE_OK;
}

tsfde_status set_mu(Problem* P, const double* mu) {
    if (!P || !mu) { set_error("set_mu: NULL argument"); return TSFDE_EINVAL; }
    if (!finite_all(mu, P->Nd)) { set_error("set_mu: non-finite value in mu"); return TSFDE_ENONFINITE; }
    try {
        P->mu_h.assign(mu, mu + P->Nd);
        TSFDE_HIP(hipMemcpy(P->d_mu, mu, sizeof(double) * P->Nd, hipMemcpyHostToDevice));
    } catch (const HipError& e) {
        set_error("set_mu: %s failed: %s", e.where.c_str(), hipGetErrorString(e.code));
        return TSFDE_EDEVICE;
    }
    return TSFDE_OK;
}

}  // namespace tsfde
