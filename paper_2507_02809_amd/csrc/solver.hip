// Operator applications and the Krylov solver behind the C ABI:
//   apply_A      z = A y (§5 'Implementation' of the matvec)
//   apply_P_inv  y = P^{-1} z by forward substitution over time (§5.1 'Implementation'),
//                diagonal blocks solved by preconditioned CG on their symmetrised form
//   gmres_solve  right-preconditioned flexible GMRES(m) with classical Gram-Schmidt done
//                twice, Givens rotations on the host in FP64; MIXED precision wraps it in
//                iterative refinement with an FP64 residual
//   recover_f    z of eq. lin-syst, solve from x0 = 0, f~ = last block (§5, §6)
//   batches      several problems side by side on worker streams (recover_f, its gradient)
//   transposed   A^T lam, P^{-T} g by backward substitution, the adjoint solve and the
//                vector-Jacobian product of f~ in mu, alpha and the gamma2 samples
//   arnoldi      the Hessenberg matrix of Arnoldi on A P^{-1} (spectral estimates)
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "grid_sync.hpp"
#include "hessenberg.hpp"
#include "internal.hpp"
#include "residency.hpp"

namespace tsfde {

tsfde_status create(int d, int N, int M, double T, double beta, double omega, double alpha, const double* gamma1,
                    const double* gamma2, const double* q, const double* rho, const double* mu, double length,
                    const double* stencil, Problem** out);
tsfde_status set_mu(Problem* P, const double* mu);
tsfde_status set_gamma2(Problem* P, const double* gamma2);
tsfde_status compute_stencil(int d, int N, double omega, double* out);
void free_problem(Problem* P);
const char* last_error();

static bool verbose() {
    static const int v = [] {
        const char* e = std::getenv("TSFDE_VERBOSE");
        return (e && *e && *e != '0') ? 1 : 0;
    }();
    return v != 0;
}

static double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
double now_seconds() { return now(); }

// FP32 diagonal-block solves cannot reach residuals much below the FP32 rounding level
constexpr double kInnerTolF32 = 1e-6;

static Opts get_opts(const tsfde_opts* o) {
    Opts r;
    if (!o) return r;
    r.restart = o->restart;
    r.maxit = o->maxit;
    r.tol = o->tol;
    r.precision = o->precision;
    r.use_precond = o->use_precond;
    r.inner_tol = o->inner_tol;
    r.inner_maxit = o->inner_maxit;
    r.refine_tol = o->refine_tol;
    r.max_refine = o->max_refine;
    r.block_solver = o->block_solver;
    r.warm_start = o->warm_start;
    r.max_device_bytes = o->max_device_bytes;
    r.recompute_z = o->recompute_z;
    r.graph = o->graph;
    return r;
}

static bool check_opts(const Opts& o) {
    if (o.restart < 1 || o.restart > kMaxRestart) { set_error("opts.restart must be in [1, 1000]"); return false; }
    if (!(o.tol > 0.0) || !(o.inner_tol > 0.0) || !(o.refine_tol > 0.0)) {
        set_error("opts tolerances must be > 0");
        return false;
    }
    if (o.inner_maxit < 1 || o.max_refine < 1) { set_error("opts.inner_maxit and max_refine must be >= 1"); return false; }
    if (o.precision != TSFDE_FP64 && o.precision != TSFDE_MIXED && o.precision != TSFDE_PREC_F32) {
        set_error("opts.precision invalid");
        return false;
    }
    if (o.warm_start < TSFDE_WARM_PREVIOUS || o.warm_start > TSFDE_WARM_HALF) {
        set_error("opts.warm_start invalid");
        return false;
    }
    if (o.block_solver != TSFDE_BLOCK_CG && o.block_solver != TSFDE_BLOCK_TAU && o.block_solver != TSFDE_BLOCK_STRANG) {
        set_error("opts.block_solver invalid");
        return false;
    }
    if (o.max_device_bytes < 0 || o.recompute_z < 0 || o.recompute_z > 1 || o.graph < 0 || o.graph > 1) {
        set_error("opts.max_device_bytes must be >= 0, opts.recompute_z and opts.graph 0 or 1");
        return false;
    }
    return true;
}

template <typename T>
static Dev<T>& dev(Problem& P);
template <>
Dev<double>& dev<double>(Problem& P) { return P.f64; }
template <>
Dev<float>& dev<float>(Problem& P) { return P.f32; }

// ---------------------------------------------------------------------------
// A y
// ---------------------------------------------------------------------------
static int env_int(const char* name, int dflt);

// d = 2 with TSFDE_MV_OVERLAP=1: the history sum (ALU-bound) runs on the problem's second stream while
// the row and column Toeplitz passes (memory- and latency-bound) run on the caller's, which waits for it
// before the epilogue adds c_t gamma2 .* B y to z.  Off by default: at N = 255, M = 256 the two
// contend for the CUs and the call takes longer (0.571 against 0.532 ms in FP64).
template <typename T>
static void apply_A_impl(Problem& P, const T* y, T* z, hipStream_t st) {
    Dev<T>& D = dev<T>(P);
    if (toeplitz2d_supported(P) && env_int("TSFDE_MV_OVERLAP", 0) != 0) {
        if (!P.mv_aux) {
            TSFDE_HIP(hipStreamCreateWithFlags(&P.mv_aux, hipStreamNonBlocking));
            TSFDE_HIP(hipEventCreateWithFlags(&P.mv_fork, hipEventDisableTiming));
            TSFDE_HIP(hipEventCreateWithFlags(&P.mv_join, hipEventDisableTiming));
        }
        TSFDE_HIP(hipEventRecord(P.mv_fork, st));
        TSFDE_HIP(hipStreamWaitEvent(P.mv_aux, P.mv_fork, 0));
        launch_history_matvec<T>(P, D, y, z, P.mv_aux);
        TSFDE_HIP(hipEventRecord(P.mv_join, P.mv_aux));
        launch_toeplitz2d_matvec<T>(P, D, y, z, st, nullptr, P.mv_join);
        return;
    }
    launch_history_matvec<T>(P, D, y, z, st);
    if (!launch_toeplitz2d_matvec<T>(P, D, y, z, st)) launch_toeplitz_matvec<T>(P, D, y, z, st);
}

// ---------------------------------------------------------------------------
// P^{-1} z by forward substitution; returns CG iterations
// ---------------------------------------------------------------------------
static int env_int(const char* name, int dflt) {
    const char* e = std::getenv(name);
    return (e && *e) ? std::atoi(e) : dflt;
}

// the tau-block form runs in the persistent kernels where they use the sine transform of size N (d = 2,
// 2(N+1) a power of two), else by dense sine-transform passes of any N; the Strang form needs its
// Hartley passes to fit the LDS and Strang's circulant of the stencil to be positive definite (its
// tables are built here on first use)
static bool tau_persistent(const Problem& P) {
    return P.d == 2 && P.tau_ok && persistent_supported(P) && env_int("TSFDE_PINV", 1) != 0;
}

static bool block_solver_supported(Problem& P, const Opts& o) {
    if (!o.use_precond || o.block_solver == TSFDE_BLOCK_CG) return true;
    if (o.block_solver == TSFDE_BLOCK_STRANG) {
        if (!strang_supported(P)) {
            set_error("opts.block_solver = TSFDE_BLOCK_STRANG: N = %d is too large for the transform passes", P.N);
            return false;
        }
        try {
            ensure_strang(P);
        } catch (const HipError& e) {
            set_error("opts.block_solver = TSFDE_BLOCK_STRANG: %s failed: %s", e.where.c_str(), hipGetErrorString(e.code));
            return false;
        }
        if (!(P.strang_min > 0.0)) {
            set_error("opts.block_solver = TSFDE_BLOCK_STRANG: Strang's circulant of the stencil is not positive "
                      "definite (smallest eigenvalue %g)", P.strang_min);
            return false;
        }
        return true;
    }
    if (tau_persistent(P)) return true;
    if (!tau_dense_supported(P)) {
        set_error("opts.block_solver = TSFDE_BLOCK_TAU: N = %d is too large for the dense sine-transform passes", P.N);
        return false;
    }
    try {
        ensure_tau_dense(P);
    } catch (const HipError& e) {
        set_error("opts.block_solver = TSFDE_BLOCK_TAU: %s failed: %s", e.where.c_str(), hipGetErrorString(e.code));
        return false;
    }
    if (!(P.taud_min > 0.0)) {
        set_error("opts.block_solver = TSFDE_BLOCK_TAU: the tau matrix of the stencil is not positive definite "
                  "(smallest eigenvalue %g)", P.taud_min);
        return false;
    }
    return true;
}

template <typename T>
static void*& pwork(Problem& P);
template <>
void*& pwork<double>(Problem& P) { return P.pw64; }
template <>
void*& pwork<float>(Problem& P) { return P.pw32; }

// multi-launch forward substitution (one kernel per CG phase, host convergence test); kept as the
// reference path and for shapes the persistent kernel does not cover
template <typename T>
static long long pinv_launch(Problem& P, const T* z, T* y, const Opts& o, hipStream_t st, bool last_block);

template <typename T>
static long long pinv_impl(Problem& P, const T* z, T* y, const Opts& o, hipStream_t st, bool last_block) {
    // TSFDE_PINV=0 selects the multi-launch path; TSFDE_PINV_BLOCKS overrides the grid size;
    // TSFDE_PINV_FIXED=0 keeps the 2D sine-transform path on its run-time-length kernel;
    // TSFDE_EXTRAP overrides opts.warm_start (the block CG's initial guess)
    if (o.block_solver == TSFDE_BLOCK_STRANG) {
        pinv_strang<T>(P, dev<T>(P), z, y, last_block, st);
        return 0;
    }
    if (o.block_solver == TSFDE_BLOCK_TAU && !tau_persistent(P)) {
        pinv_tau_dense<T>(P, dev<T>(P), z, y, last_block, st);
        return 0;
    }
    if (env_int("TSFDE_PINV", 1) != 0 && persistent_supported(P)) {
        set_persistent_blocks(env_int("TSFDE_PINV_BLOCKS", -1));
        set_persistent_fixed_length(env_int("TSFDE_PINV_FIXED", 1) != 0);
        return pinv_persistent_run<T>(P, dev<T>(P), pwork<T>(P), z, y, o.inner_tol, o.inner_maxit, last_block,
                                      env_int("TSFDE_EXTRAP", o.warm_start), o.block_solver == TSFDE_BLOCK_TAU ? 1 : 0,
                                      st);
    }
    return pinv_launch<T>(P, z, y, o, st, last_block);
}

// One diagonal block by preconditioned CG, one kernel launch per CG phase and the convergence test on
// the host: (dg + c B) x = rhs (dg null: c B x = rhs) from the initial x, to relative residual
// inner_tol; the preconditioner is the tau matrix (sigma I + c tau(B)) when the sine transform is
// available, else the diagonal.  Returns the CG iterations.
template <typename T>
static long long block_cg(Problem& P, Dev<T>& D, const T* rhs, T* x, const T* dg, T c, T sigma, const Opts& o,
                          hipStream_t st) {
    const long long Nd = P.Nd;
    T* r = D.pcg + Nd;
    T* zz = D.pcg + 2 * Nd;
    T* p = D.pcg + 3 * Nd;
    T* q = D.pcg + 4 * Nd;
    double* scal = P.dev_scalars;
    double* hs = P.host_scalars;
    const double tol2 = o.inner_tol * o.inner_tol;
    long long total = 0;
    int np = 0;
    auto prec = [&](const T* rin, T* zout) {
        if (P.tau_ok) launch_tau_prec<T>(P, D, rin, zout, sigma, c, D.partial, &np, st);
        else launch_jacobi_prec<T>(rin, zout, dg, c, T(P.a0), Nd, D.partial, &np, st);
    };
    // r = rhs - A_s x ; ||r||^2 ; ||rhs||^2
    launch_spd_apply<T>(P, D, x, q, dg, c, D.partial, &np, st);
    launch_sub_partials<T>(rhs, q, r, Nd, D.partial, &np, st);
    launch_sum_partials(D.partial, np, scal + 3, st);
    launch_dot_partials<T>(rhs, rhs, Nd, D.partial, &np, st);
    launch_sum_partials(D.partial, np, scal + 8, st);
    TSFDE_HIP(hipMemcpyAsync(hs, scal, 16 * sizeof(double), hipMemcpyDeviceToHost, st));
    TSFDE_HIP(hipStreamSynchronize(st));
    const double bb = hs[8];
    double rr = hs[3];
    if (!(bb > 0.0)) {
        launch_fill(x, Nd, T(0), st);
    } else if (rr > tol2 * bb) {
        prec(r, zz);
        launch_sum_partials(D.partial, np, scal + 0, st);
        launch_copy<T>(zz, p, Nd, st);
        for (int it = 1; it <= o.inner_maxit; ++it) {
            launch_spd_apply<T>(P, D, p, q, dg, c, D.partial, &np, st);
            launch_sum_partials(D.partial, np, scal + 1, st);
            launch_cg_scalars(scal, 0, st);
            launch_cg_update_xr<T>(x, r, p, q, scal, Nd, D.partial, &np, st);
            launch_sum_partials(D.partial, np, scal + 3, st);
            TSFDE_HIP(hipMemcpyAsync(hs + 3, scal + 3, sizeof(double), hipMemcpyDeviceToHost, st));
            TSFDE_HIP(hipStreamSynchronize(st));
            ++total;
            rr = hs[3];
            if (rr <= tol2 * bb || !std::isfinite(rr)) break;
            prec(r, zz);
            launch_sum_partials(D.partial, np, scal + 5, st);
            launch_cg_scalars(scal, 1, st);
            launch_cg_update_p<T>(p, zz, scal, Nd, st);
        }
    }
    return total;
}

template <typename T>
static long long pinv_launch(Problem& P, const T* z, T* y, const Opts& o, hipStream_t st, bool last_block) {
    Dev<T>& D = dev<T>(P);
    const long long Nd = P.Nd;
    T* x = D.pcg;
    T* rhs = x + 7 * Nd;
    long long total = 0;
    const int last = last_block ? P.M : P.M - 1;
    for (int s = 0; s <= last; ++s) {
        launch_step_rhs<T>(P, D, z, y, s, rhs, T(P.cf), st);
        const T* dg = (s < P.M) ? D.dg + (long long)s * Nd : nullptr;
        const T c = (s < P.M) ? T(P.ct) : T(1);
        const T sigma = (s < P.M) ? T(P.sigma[s]) : T(0);
        if (s > 0 && s < P.M) launch_copy<T>(y + (long long)(s - 1) * Nd, x, Nd, st);
        else launch_fill(x, Nd, T(0), st);
        total += block_cg<T>(P, D, rhs, x, dg, c, sigma, o, st);
        launch_copy<T>(x, y + (long long)s * Nd, Nd, st);
    }
    return total;
}

// ---------------------------------------------------------------------------
// Transposed problem: A^T lam and P^{-T} g (FP64)
// ---------------------------------------------------------------------------
static void apply_AT_impl(Problem& P, const double* lam, double* z, hipStream_t st) {
    Dev<double>& D = P.f64;
    if (!P.adj_u) dev_alloc(P, P.adj_u, P.ntot);
    launch_scale_g2<double>(P, D, lam, P.adj_u, -1, false, st);
    launch_history_adj<double>(P, D, lam, z, st);
    // B products of the gamma2-scaled slices added with weight c_t (c_f for the last); the last
    // slice keeps its f-row terms (ylast = z^(M) itself)
    Dev<double> Dn = D;
    Dn.gamma2 = nullptr;
    const double* ylast = z + (size_t)P.M * P.Nd;
    if (!launch_toeplitz2d_matvec<double>(P, Dn, P.adj_u, z, st, ylast))
        launch_toeplitz_matvec<double>(P, Dn, P.adj_u, z, st, ylast);
}

// lam = P^{-T} g by backward substitution over the block rows of P^T (block upper triangular): block
// m solves (e_0 D_1 + c_t B D_2) lam^(m) = r, i.e. the SPD system (dg + c_t B) u = r for u = D_2 lam^(m)
// (the last block: c_f B D_2^(M-1) lam^(M) = g^(M)).  Returns CG iterations.
static long long ptinv_launch(Problem& P, const double* g, double* lam, const Opts& o, hipStream_t st) {
    Dev<double>& D = P.f64;
    const long long Nd = P.Nd;
    double* x = D.pcg;
    double* rhs = x + 7 * Nd;
    long long total = 0;
    // the block rows m < M on the persistent kernels (TSFDE_PTINV=0 keeps them on this loop): after the
    // last block row, the transposed sweep in reversed step order
    const bool pers = env_int("TSFDE_PTINV", 1) != 0 && env_int("TSFDE_PINV", 1) != 0 && persistent_supported(P);
    if (pers) {
        launch_adj_step_rhs<double>(P, D, g, lam, P.M, rhs, st);
        launch_fill(x, Nd, 0.0, st);
        total += block_cg<double>(P, D, rhs, x, nullptr, 1.0, 0.0, o, st);
        launch_scale_g2<double>(P, D, x, lam, P.M, true, st);
        const size_t MN = (size_t)P.M * Nd;
        if (!P.adj_rev) dev_alloc(P, P.adj_rev, 2 * MN + (size_t)P.M);
        double* zrev = P.adj_rev;
        double* dgrev = P.adj_rev + MN;
        double* sigrev = P.adj_rev + 2 * MN;
        std::vector<double> sr(P.M);
        for (int k = 0; k < P.M; ++k) sr[k] = P.sigma[P.M - 1 - k];
        TSFDE_HIP(hipMemcpyAsync(sigrev, sr.data(), sizeof(double) * P.M, hipMemcpyHostToDevice, st));
        launch_adj_reverse(P, g, lam, zrev, dgrev, st);
        total += pinv_adjoint_run(P, zrev, dgrev, sigrev, lam, o.inner_tol, o.inner_maxit,
                                  env_int("TSFDE_EXTRAP", o.warm_start), st);  // synchronises st
        launch_adj_unreverse(P, lam, st);
        return total;
    }
    for (int m = P.M; m >= 0; --m) {
        launch_adj_step_rhs<double>(P, D, g, lam, m, rhs, st);
        const double* dg = (m < P.M) ? D.dg + (long long)m * Nd : nullptr;
        const double c = (m < P.M) ? P.ct : 1.0;
        const double sigma = (m < P.M) ? P.sigma[m] : 0.0;
        if (m >= P.M - 1) launch_fill(x, Nd, 0.0, st);  // else warm start from u of block m + 1
        total += block_cg<double>(P, D, rhs, x, dg, c, sigma, o, st);
        launch_scale_g2<double>(P, D, x, lam, m, true, st);
    }
    return total;
}

// ---------------------------------------------------------------------------
// FGMRES (FP64 Arnoldi), operators given as callbacks on FP64 vectors
// ---------------------------------------------------------------------------

// The Krylov basis V (m + 1 vectors) and the preconditioned directions Z (m vectors, or one when they
// are recomputed at the end of each cycle instead of kept).  With a cap on the problem's device memory
// (opts.max_device_bytes, 0 = none) Z is recomputed when keeping it would exceed the cap, and a basis
// that does not fit even then is refused.  Returns whether Z is recomputed.
static bool ensure_basis(Problem& P, int m, const Opts& o) {
    const size_t vec = sizeof(double) * (size_t)P.ntot;
    const size_t base = P.bytes - P.basis_bytes;  // the problem's other arrays
    bool recompute = o.recompute_z != 0;
    if (o.max_device_bytes > 0) {
        const size_t cap = (size_t)o.max_device_bytes;
        if (!recompute && base + (size_t)(2 * m + 1) * vec > cap) recompute = true;
        if (base + (size_t)(m + 2) * vec > cap) {
            char buf[256];
            std::snprintf(buf, sizeof(buf),
                          "max_device_bytes = %lld: the problem holds %zu bytes and the Krylov basis of restart %d needs "
                          "at least %zu more (Z recomputed)",
                          o.max_device_bytes, base, m, (size_t)(m + 2) * vec);
            throw CapError{buf};
        }
    }
    const int zm = recompute ? 1 : m;
    if (P.basis_m >= m && P.basis_zm >= zm) return recompute;
    if (P.V) (void)hipFree(P.V);
    if (P.Z) (void)hipFree(P.Z);
    P.V = P.Z = nullptr;
    P.basis_m = P.basis_zm = 0;
    P.bytes -= P.basis_bytes;
    P.basis_bytes = 0;
    dev_alloc(P, P.V, (size_t)(m + 1) * P.ntot);
    P.basis_bytes += (size_t)(m + 1) * vec;
    dev_alloc(P, P.Z, (size_t)zm * P.ntot);
    P.basis_bytes += (size_t)zm * vec;
    P.basis_m = m;
    P.basis_zm = zm;
    return recompute;
}

// h = V[0..k)^T w, in chunks of at most kArnMaxK basis vectors
static void arn_dot(const double* V, long long n, int k, const double* w, double* partials, int nblk, double* h,
                    hipStream_t st) {
    for (int c0 = 0; c0 < k; c0 += kArnMaxK) {
        const int kc = std::min(kArnMaxK, k - c0);
        launch_multidot(V + (size_t)c0 * n, n, kc, w, partials, nblk, st);
        launch_multidot_finish(partials, nblk, kc, h + c0, st);
    }
}

// w -= V[0..k) h; the partials then hold the block sums of w . w
static void arn_sub_norm(const double* V, long long n, int k, const double* h, double* w, double* partials, int nblk,
                         hipStream_t st) {
    for (int c0 = 0; c0 < k; c0 += kArnMaxK)
        launch_cgs_sub_norm(V + (size_t)c0 * n, n, std::min(kArnMaxK, k - c0), h + c0, w, partials, nblk, st);
}

// Classical Gram-Schmidt of w against V[0..k), repeated once (h1 then h2, the coefficients of the two
// passes; w ends orthogonal to V and unnormalised, nrm2 = ||w||^2).  Three sweeps over V when k fits
// one pass of the fused kernels.
static void cgs2(const double* V, long long n, int k, double* w, double* partials, int nblk, double* h1, double* h2,
                 double* nrm2, hipStream_t st) {
    arn_dot(V, n, k, w, partials, nblk, h1, st);
    if (k <= kArnMaxK) {
        launch_cgs_sub_dot(V, n, k, h1, w, partials, nblk, st);
        launch_multidot_finish(partials, nblk, k, h2, st);
    } else {
        arn_sub_norm(V, n, k, h1, w, partials, nblk, st);
        arn_dot(V, n, k, w, partials, nblk, h2, st);
    }
    arn_sub_norm(V, n, k, h2, w, partials, nblk, st);
    launch_multidot_finish(partials, nblk, 1, nrm2, st);
}

static double dev_dot(Problem& P, const double* a, const double* b, long long n, hipStream_t st) {
    int np = 0;
    launch_dot_partials<double>(a, b, n, P.f64.partial, &np, st);
    launch_sum_partials(P.f64.partial, np, P.dev_scalars + 16, st);
    TSFDE_HIP(hipMemcpyAsync(P.host_scalars + 16, P.dev_scalars + 16, sizeof(double), hipMemcpyDeviceToHost, st));
    TSFDE_HIP(hipStreamSynchronize(st));
    return P.host_scalars[16];
}

// Solves A x = b to ||b - A x|| <= rtol * ||b|| (estimated from the Arnoldi least-squares residual,
// checked exactly at each restart).  x holds the initial guess.  r_work: n_tot scratch.
// Returns the number of Arnoldi steps; *conv set when the tolerance was met.
static int fgmres(Problem& P, const SolveOps& ops, const double* b, double* x, double* r_work, double rtol,
                  int restart, int maxit, hipStream_t st, tsfde_stats& S, bool& conv, double& relres,
                  bool exact_final, const Opts& o) {
    const long long n = P.ntot;
    const bool recompute = ensure_basis(P, restart, o);
    const int nblk = kArnBlocks;
    if (!P.arn_part) dev_alloc(P, P.arn_part, kArnBlocks * kArnMaxK);
    if (!P.arn_h) dev_alloc(P, P.arn_h, (2 * (kMaxRestart + 2) + 1));
    double* partials = P.arn_part;
    // hbuf: first-pass coefficients [0, restart + 2), second-pass ones [hs, 2 hs), then ||w||^2
    const int hs = restart + 2;
    double* hbuf = P.arn_h;
    std::vector<double> Hc((size_t)(restart + 1) * restart, 0.0), cs(restart), sn(restart), g(restart + 1), yk(restart);
    std::vector<double> hhost(2 * hs + 1);
    const double bnorm = std::sqrt(dev_dot(P, b, b, n, st));
    int its = 0;
    conv = false;
    relres = 1.0;
    if (!(bnorm > 0.0)) {
        launch_fill(x, n, 0.0, st);
        conv = true;
        relres = 0.0;
        return 0;
    }
    while (true) {
        double t0 = now();
        ops.A(x, r_work);
        TSFDE_HIP(hipStreamSynchronize(st));
        S.t_matvec += now() - t0;
        launch_axpby(1.0, b, -1.0, r_work, r_work, n, st);
        const double beta = std::sqrt(dev_dot(P, r_work, r_work, n, st));
        relres = beta / bnorm;
        P.res_hist.push_back(relres);
        if (verbose())
            std::fprintf(stderr, "[tsfde] fgmres its=%d restarts=%d true relres=%.3e (target %.1e)\n", its, S.restarts,
                         relres, rtol);
        if (relres <= rtol) { conv = true; break; }
        if (its >= maxit) break;
        const int m = std::min(restart, maxit - its);
        launch_axpby(1.0 / beta, r_work, 0.0, r_work, P.V, n, st);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        bool lucky = false;
        for (int j = 0; j < m; ++j) {
            double* vj = P.V + (size_t)j * n;
            double* zj = P.Z + (size_t)(recompute ? 0 : j) * n;
            double* w = P.V + (size_t)(j + 1) * n;
            t0 = now();
            S.inner_iters += ops.M(vj, zj);
            TSFDE_HIP(hipStreamSynchronize(st));
            S.t_precond += now() - t0;
            t0 = now();
            ops.A(zj, w);
            TSFDE_HIP(hipStreamSynchronize(st));
            S.t_matvec += now() - t0;
            t0 = now();
            // classical Gram-Schmidt, twice
            cgs2(P.V, n, j + 1, w, partials, nblk, hbuf, hbuf + hs, hbuf + 2 * hs, st);
            TSFDE_HIP(hipMemcpyAsync(hhost.data(), hbuf, sizeof(double) * (2 * hs + 1), hipMemcpyDeviceToHost, st));
            TSFDE_HIP(hipStreamSynchronize(st));
            const double hn = std::sqrt(hhost[2 * hs]);
            for (int i = 0; i <= j; ++i) Hc[(size_t)i * restart + j] = hhost[i] + hhost[hs + i];
            Hc[(size_t)(j + 1) * restart + j] = hn;
            if (hn > 0.0) launch_axpby(1.0 / hn, w, 0.0, w, w, n, st);
            S.t_ortho += now() - t0;
            // Givens on column j
            for (int i = 0; i < j; ++i) {
                const double a = Hc[(size_t)i * restart + j], bq = Hc[(size_t)(i + 1) * restart + j];
                Hc[(size_t)i * restart + j] = cs[i] * a + sn[i] * bq;
                Hc[(size_t)(i + 1) * restart + j] = -sn[i] * a + cs[i] * bq;
            }
            const double a = Hc[(size_t)j * restart + j], bq = Hc[(size_t)(j + 1) * restart + j];
            const double rr = std::hypot(a, bq);
            cs[j] = rr > 0.0 ? a / rr : 1.0;
            sn[j] = rr > 0.0 ? bq / rr : 0.0;
            Hc[(size_t)j * restart + j] = rr;
            Hc[(size_t)(j + 1) * restart + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            ++its;
            ++S.iters;
            P.res_hist.push_back(std::fabs(g[j + 1]) / bnorm);
            if (verbose())
                std::fprintf(stderr, "[tsfde]   it=%d est relres=%.3e inner=%lld\n", its, std::fabs(g[j + 1]) / bnorm,
                             (long long)S.inner_iters);
            if (std::fabs(g[j + 1]) <= rtol * bnorm) break;
            if (hn == 0.0) { lucky = true; break; }
        }
        (void)lucky;
        // y = R^{-1} g, x += Z y
        for (int i = k - 1; i >= 0; --i) {
            double acc = g[i];
            for (int l = i + 1; l < k; ++l) acc -= Hc[(size_t)i * restart + l] * yk[l];
            yk[i] = acc / Hc[(size_t)i * restart + i];
        }
        if (recompute) {
            // z_j = M v_j again (the preconditioner is a deterministic function of its input, so the
            // same directions come back), x += y_j z_j one at a time
            for (int j = 0; j < k; ++j) {
                double t0r = now();
                S.inner_iters += ops.M(P.V + (size_t)j * n, P.Z);
                TSFDE_HIP(hipStreamSynchronize(st));
                S.t_precond += now() - t0r;
                launch_axpby(yk[j], P.Z, 1.0, x, x, n, st);
            }
            TSFDE_HIP(hipStreamSynchronize(st));
        } else {
            TSFDE_HIP(hipMemcpyAsync(hbuf, yk.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
            double t0u = now();
            launch_gemv_add(P.Z, n, k, hbuf, x, st);
            TSFDE_HIP(hipStreamSynchronize(st));
            S.t_ortho += now() - t0u;
        }
        const double est = std::fabs(g[k]) / bnorm;
        if (est <= rtol && !exact_final) {
            relres = est;
            conv = true;
            break;
        }
        ++S.restarts;
    }
    return its;
}

// Restart cycles as HIP graphs: the path applies when P^{-1} is the persistent forward substitution
// (or absent) and the directions z_j are kept.
static bool graph_supported(Problem& P, const Opts& o) {
    if (o.recompute_z) return false;
    if (!o.use_precond) return true;
    if (env_int("TSFDE_PINV", 1) == 0 || !persistent_supported(P)) return false;
    return o.block_solver == TSFDE_BLOCK_CG || (o.block_solver == TSFDE_BLOCK_TAU && tau_persistent(P));
}

// FGMRES(m) whose restart cycles run as one HIP graph each.  Per cycle, on the host: r = b - A x and
// its norm (the true residual, the convergence test); then the graph, captured once per problem and
// settings and replayed for every later cycle and solve: v_0 = r / ||r||, and m Arnoldi steps
// z_j = M v_j, w = A z_j, classical Gram-Schmidt twice (coefficients and ||w||^2 into the device
// array cyc_h, column j), v_{j+1} = w / ||w|| by the device-side norm, the coefficients copied to
// pinned host memory at the end.  The host applies the Givens rotations, takes the first k <= m
// steps whose least-squares residual meets rtol and adds Z y to x.  A breakdown (||w|| = 0) zeroes
// the later directions, which the host never uses.
static int fgmres_graph(Problem& P, const std::function<SolveOps(hipStream_t)>& make_ops, const double* b, double* x,
                        double* r_work, double rtol, int m, int maxit, hipStream_t st, tsfde_stats& S, bool& conv,
                        double& relres, const Opts& o) {
    const long long n = P.ntot;
    ensure_basis(P, m, o);
    const int nblk = kArnBlocks;
    if (!P.arn_part) dev_alloc(P, P.arn_part, kArnBlocks * kArnMaxK);
    if (!P.arn_h) dev_alloc(P, P.arn_h, (2 * (kMaxRestart + 2) + 1));
    const int hs = m + 2, stride = 2 * hs + 1;
    const int len = m * stride + 1;  // the last slot: ||r||^2 of the cycle's start
    if (P.cyc_len < len) {
        if (P.cyc_h) (void)hipFree(P.cyc_h);
        if (P.cyc_h_host) (void)hipHostFree(P.cyc_h_host);
        P.cyc_h = nullptr;
        P.cyc_h_host = nullptr;
        P.cyc_len = 0;
        TSFDE_HIP(hipMalloc(&P.cyc_h, sizeof(double) * len));
        TSFDE_HIP(hipHostMalloc(&P.cyc_h_host, sizeof(double) * len, hipHostMallocDefault));
        P.cyc_len = len;
        if (P.cyc_exec) (void)hipGraphExecDestroy(P.cyc_exec);
        P.cyc_exec = nullptr;
    }
    if (!P.cyc_stream) TSFDE_HIP(hipStreamCreateWithFlags(&P.cyc_stream, hipStreamNonBlocking));
    double* beta2 = P.cyc_h + (size_t)m * stride;
    const bool f32 = o.precision == TSFDE_PREC_F32;
    const SolveOps ops = make_ops(st);
    // what the captured cycle depends on
    unsigned long long key[10];
    {
        double it = o.inner_tol;
        unsigned long long itb = 0;
        std::memcpy(&itb, &it, sizeof(itb));
        key[0] = (unsigned long long)m;
        key[1] = (unsigned long long)(uintptr_t)P.V;
        key[2] = (unsigned long long)(uintptr_t)P.Z;
        key[3] = (unsigned long long)(uintptr_t)r_work;
        key[4] = (unsigned long long)(uintptr_t)P.cyc_h;
        key[5] = itb;
        key[6] = ((unsigned long long)o.block_solver << 32) | (unsigned)o.inner_maxit;
        key[7] = ((unsigned long long)o.warm_start << 32) | (unsigned)o.precision;
        key[8] = ((unsigned long long)o.use_precond << 32) | (unsigned)(P.mv_variant + 1);
        key[9] = ((unsigned long long)(unsigned)P.pinv_blocks << 32) | (unsigned)(shared_launch() ? 1 : 0);
    }
    const double bnorm = std::sqrt(dev_dot(P, b, b, n, st));
    conv = false;
    relres = 1.0;
    if (!(bnorm > 0.0)) {
        launch_fill(x, n, 0.0, st);
        conv = true;
        relres = 0.0;
        return 0;
    }
    std::vector<double> Hc((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), yk(m);
    int its = 0;
    bool warmed = P.cyc_exec != nullptr;
    while (true) {
        double t0 = now();
        ops.A(x, r_work);
        launch_axpby(1.0, b, -1.0, r_work, r_work, n, st);
        int np = 0;
        launch_dot_partials<double>(r_work, r_work, n, P.f64.partial, &np, st);
        launch_sum_partials(P.f64.partial, np, beta2, st);
        TSFDE_HIP(hipMemcpyAsync(P.host_scalars + 16, beta2, sizeof(double), hipMemcpyDeviceToHost, st));
        TSFDE_HIP(hipStreamSynchronize(st));
        S.t_matvec += now() - t0;
        const double beta = std::sqrt(std::max(0.0, P.host_scalars[16]));
        relres = beta / bnorm;
        P.res_hist.push_back(relres);
        if (relres <= rtol) { conv = true; break; }
        if (its >= maxit) break;
        if (!P.cyc_exec || std::memcmp(key, P.cyc_key, sizeof(key)) != 0) {
            if (!warmed) {
                // one preconditioner application outside the capture: work buffers and tables are
                // allocated on first use
                ops.M(r_work, P.Z);
                TSFDE_HIP(hipStreamSynchronize(st));
                warmed = true;
            }
            if (P.cyc_exec) (void)hipGraphExecDestroy(P.cyc_exec);
            P.cyc_exec = nullptr;
            const SolveOps gops = make_ops(P.cyc_stream);
            hipStream_t cs_ = P.cyc_stream;
            P.graph_slots = 0;
            P.capturing = true;
            struct Uncapture {  // capture mode ends however the capture ends
                Problem& P;
                hipStream_t s;
                bool open = true;
                ~Uncapture() {
                    P.capturing = false;
                    if (open) {
                        hipGraph_t gr = nullptr;
                        (void)hipStreamEndCapture(s, &gr);
                        if (gr) (void)hipGraphDestroy(gr);
                    }
                }
            } unc{P, cs_};
            TSFDE_HIP(hipStreamBeginCapture(cs_, hipStreamCaptureModeThreadLocal));
            launch_copy<double>(r_work, P.V, n, cs_);
            launch_scale_rsqrt(P.V, n, beta2, cs_);
            for (int j = 0; j < m; ++j) {
                double* vj = P.V + (size_t)j * n;
                double* zj = P.Z + (size_t)j * n;
                double* w = P.V + (size_t)(j + 1) * n;
                double* hj = P.cyc_h + (size_t)j * stride;
                gops.M(vj, zj);
                gops.A(zj, w);
                cgs2(P.V, n, j + 1, w, P.arn_part, nblk, hj, hj + hs, hj + 2 * hs, cs_);
                launch_scale_rsqrt(w, n, hj + 2 * hs, cs_);
            }
            TSFDE_HIP(hipMemcpyAsync(P.cyc_h_host, P.cyc_h, sizeof(double) * len, hipMemcpyDeviceToHost, cs_));
            hipGraph_t graph = nullptr;
            unc.open = false;
            TSFDE_HIP(hipStreamEndCapture(cs_, &graph));
            hipGraphExec_t exec = nullptr;
            const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            TSFDE_HIP(ie);
            P.cyc_exec = exec;
            std::memcpy(P.cyc_key, key, sizeof(key));
        }
        // replay, the persistent grids' CU slots held around it
        t0 = now();
        long long inner = 0;
        {
            int dev = 0, ncu = 0;
            TSFDE_HIP(hipGetDevice(&dev));
            TSFDE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
            ResidencyTicket ticket;
            struct Release {
                ResidencyTicket& t;
                ~Release() { t.release(); }
            } rel{ticket};
            const bool pers = o.use_precond && P.graph_slots > 0;
            if (pers) {
                pinv_graph_prepare(P, f32, st);
                ticket.hold(&residency_budget(dev, ncu), P.graph_slots);
            }
            TSFDE_HIP(hipGraphLaunch(P.cyc_exec, st));
            TSFDE_HIP(hipStreamSynchronize(st));
            if (pers) inner = pinv_graph_finish(P, f32, st);
        }
        S.t_precond += now() - t0;  // the whole cycle (P^{-1} dominates it)
        S.inner_iters += inner;
        // Givens on the host over the cycle's coefficients, up to the first step that meets rtol
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        const double* hh = P.cyc_h_host;
        int k = 0;
        for (int j = 0; j < m && its < maxit; ++j) {
            const double* hj = hh + (size_t)j * stride;
            const double nrm2 = hj[2 * hs];
            const double hn = (nrm2 > 0.0 && std::isfinite(nrm2)) ? std::sqrt(nrm2) : 0.0;
            for (int i = 0; i <= j; ++i) Hc[(size_t)i * m + j] = hj[i] + hj[hs + i];
            Hc[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = Hc[(size_t)i * m + j], bq = Hc[(size_t)(i + 1) * m + j];
                Hc[(size_t)i * m + j] = cs[i] * a + sn[i] * bq;
                Hc[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bq;
            }
            const double a = Hc[(size_t)j * m + j], bq = Hc[(size_t)(j + 1) * m + j];
            const double rr = std::hypot(a, bq);
            cs[j] = rr > 0.0 ? a / rr : 1.0;
            sn[j] = rr > 0.0 ? bq / rr : 0.0;
            Hc[(size_t)j * m + j] = rr;
            Hc[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            ++its;
            ++S.iters;
            P.res_hist.push_back(std::fabs(g[j + 1]) / bnorm);
            if (std::fabs(g[j + 1]) <= rtol * bnorm || hn == 0.0) break;
        }
        for (int i = k - 1; i >= 0; --i) {
            double acc = g[i];
            for (int l = i + 1; l < k; ++l) acc -= Hc[(size_t)i * m + l] * yk[l];
            yk[i] = Hc[(size_t)i * m + i] != 0.0 ? acc / Hc[(size_t)i * m + i] : 0.0;
        }
        TSFDE_HIP(hipMemcpyAsync(P.arn_h, yk.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
        launch_gemv_add(P.Z, n, k, P.arn_h, x, st);
        TSFDE_HIP(hipStreamSynchronize(st));
        ++S.restarts;
    }
    return its;
}

// k steps of Arnoldi (classical Gram-Schmidt twice) on the right-preconditioned operator A M from b;
// H receives the (k+1) x k Hessenberg matrix row-major (host).  Returns the steps taken (fewer than k
// on an exact breakdown).  The eigenvalues of its leading square part are Ritz values of A M, i.e.
// of M A (the same spectrum).
static int arnoldi_impl(Problem& P, const SolveOps& ops, const double* b, int k, double* H, hipStream_t st) {
    const long long n = P.ntot;
    Opts keep;  // Arnoldi keeps every direction z_j
    ensure_basis(P, k, keep);
    const int nblk = kArnBlocks;
    if (!P.arn_part) dev_alloc(P, P.arn_part, kArnBlocks * kArnMaxK);
    if (!P.arn_h) dev_alloc(P, P.arn_h, (2 * (kMaxRestart + 2) + 1));
    const int hs = k + 2;
    double* hbuf = P.arn_h;
    std::vector<double> hhost(2 * hs + 1);
    std::fill(H, H + (size_t)(k + 1) * k, 0.0);
    const double bnorm = std::sqrt(dev_dot(P, b, b, n, st));
    if (!(bnorm > 0.0)) return 0;
    launch_axpby(1.0 / bnorm, b, 0.0, b, P.V, n, st);
    for (int j = 0; j < k; ++j) {
        double* vj = P.V + (size_t)j * n;
        double* zj = P.Z + (size_t)j * n;
        double* w = P.V + (size_t)(j + 1) * n;
        ops.M(vj, zj);
        ops.A(zj, w);
        cgs2(P.V, n, j + 1, w, P.arn_part, nblk, hbuf, hbuf + hs, hbuf + 2 * hs, st);
        TSFDE_HIP(hipMemcpyAsync(hhost.data(), hbuf, sizeof(double) * (2 * hs + 1), hipMemcpyDeviceToHost, st));
        TSFDE_HIP(hipStreamSynchronize(st));
        const double hn = std::sqrt(hhost[2 * hs]);
        for (int i = 0; i <= j; ++i) H[(size_t)i * k + j] = hhost[i] + hhost[hs + i];
        H[(size_t)(j + 1) * k + j] = hn;
        if (!(hn > 0.0)) return j + 1;
        launch_axpby(1.0 / hn, w, 0.0, w, w, n, st);
    }
    return k;
}

static tsfde_status solve(Problem& P, const double* b, double* x, const Opts& o, tsfde_stats& S, hipStream_t st) {
    const long long n = P.ntot;
    const int maxit = o.maxit > 0 ? o.maxit : (int)std::min<long long>(n, 1000);
    const double t_start = now();
    P.res_hist.clear();
    struct History {  // the stats point at the problem's history however the solve ends
        Problem& P;
        tsfde_stats& S;
        ~History() {
            S.history_len = (int)P.res_hist.size();
            S.history = P.res_hist.data();
        }
    } hist{P, S};
    if (o.precision == TSFDE_FP64 || o.precision == TSFDE_PREC_F32) {
        Opts o32 = o;
        o32.inner_tol = std::max(o.inner_tol, kInnerTolF32);
        Dev<float>& F = P.f32;
        if (o.precision == TSFDE_PREC_F32 && !F.vecA) {
            dev_alloc(P, F.vecA, n);
            dev_alloc(P, F.vecB, n);
        }
        // the two operators on stream s (the graph path captures them on a stream of its own)
        auto make_ops = [&P, &o, &o32, &F, n](hipStream_t s) {
            SolveOps ops;
            ops.A = [&P, s](const double* v, double* out) { apply_A_impl<double>(P, v, out, s); };
            ops.M = [&P, &o, &o32, &F, n, s](const double* v, double* out) -> long long {
                if (!o.use_precond) { launch_copy<double>(v, out, n, s); return 0; }
                if (o.precision == TSFDE_FP64) return pinv_impl<double>(P, v, out, o, s, true);
                // FP32 preconditioner inside the FP64 flexible Krylov solve
                launch_d2f(v, F.vecA, n, s);
                const long long it = pinv_impl<float>(P, F.vecA, F.vecB, o32, s, true);
                launch_f2d(F.vecB, out, n, s);
                return it;
            };
            return ops;
        };
        if (!P.rwork) dev_alloc(P, P.rwork, n);
        bool conv = false;
        double rel = 1.0;
        if (o.graph && graph_supported(P, o))
            fgmres_graph(P, make_ops, b, x, P.rwork, o.tol, o.restart, maxit, st, S, conv, rel, o);
        else
            fgmres(P, make_ops(st), b, x, P.rwork, o.tol, o.restart, maxit, st, S, conv, rel, true, o);
        S.refinements = 1;
        S.converged = conv ? 1 : 0;
        S.rel_res = rel;
    } else {
        // iterative refinement: r = b - A x in FP64; inner FGMRES with FP32 operators on A d = r
        Dev<float>& F = P.f32;
        if (!F.vecA) {
            dev_alloc(P, F.vecA, n);
            dev_alloc(P, F.vecB, n);
        }
        SolveOps ops;
        ops.A = [&](const double* v, double* out) {
            launch_d2f(v, F.vecA, n, st);
            apply_A_impl<float>(P, F.vecA, F.vecB, st);
            launch_f2d(F.vecB, out, n, st);
        };
        Opts o32 = o;
        o32.inner_tol = std::max(o.inner_tol, kInnerTolF32);
        ops.M = [&](const double* v, double* out) -> long long {
            if (!o.use_precond) { launch_copy<double>(v, out, n, st); return 0; }
            launch_d2f(v, F.vecA, n, st);
            long long it = pinv_impl<float>(P, F.vecA, F.vecB, o32, st, true);
            launch_f2d(F.vecB, out, n, st);
            return it;
        };
        if (!P.refine_work) dev_alloc(P, P.refine_work, 3 * (size_t)n);
        double* r = P.refine_work;
        double* d = r + n;
        double* rw = r + 2 * n;
        const double bnorm = std::sqrt(dev_dot(P, b, b, n, st));
        double rel = 1.0;
        S.converged = 0;
        int used = 0;
        // every correction is followed by a residual check: at most max_refine corrections, and the
        // stats always describe the returned x
        for (int ref = 0;; ++ref) {
            double t0 = now();
            apply_A_impl<double>(P, x, r, st);
            TSFDE_HIP(hipStreamSynchronize(st));
            S.t_matvec += now() - t0;
            launch_axpby(1.0, b, -1.0, r, r, n, st);
            const double rn = std::sqrt(dev_dot(P, r, r, n, st));
            rel = bnorm > 0.0 ? rn / bnorm : 0.0;
            if (rel <= o.tol) { S.converged = 1; break; }
            if (ref >= o.max_refine || used >= maxit) break;
            launch_fill(d, n, 0.0, st);
            bool conv = false;
            double rr = 1.0;
            used += fgmres(P, ops, r, d, rw, std::max(o.refine_tol, 0.5 * o.tol / std::max(rel, 1e-300)), o.restart,
                           maxit - used, st, S, conv, rr, false, o);
            launch_axpby(1.0, x, 1.0, d, x, n, st);
            ++S.refinements;
        }
        S.rel_res = rel;
    }
    TSFDE_HIP(hipStreamSynchronize(st));
    S.t_total = now() - t_start;
    return S.converged ? TSFDE_OK : TSFDE_ENOCONV;
}

// A^T lam = g by FGMRES right-preconditioned with P^{-T} (FP64; block solves by CG to inner_tol);
// lam holds the initial guess
static tsfde_status adjoint_impl(Problem& P, const double* g, double* lam, const Opts& o, tsfde_stats& S,
                                 hipStream_t st) {
    const long long n = P.ntot;
    const int maxit = o.maxit > 0 ? o.maxit : (int)std::min<long long>(n, 1000);
    const double t_start = now();
    P.res_hist.clear();
    struct History {
        Problem& P;
        tsfde_stats& S;
        ~History() {
            S.history_len = (int)P.res_hist.size();
            S.history = P.res_hist.data();
        }
    } hist{P, S};
    SolveOps ops;
    ops.A = [&](const double* v, double* out) { apply_AT_impl(P, v, out, st); };
    ops.M = [&](const double* v, double* out) -> long long {
        if (!o.use_precond) {
            launch_copy<double>(v, out, n, st);
            return 0;
        }
        return ptinv_launch(P, v, out, o, st);
    };
    if (!P.rwork) dev_alloc(P, P.rwork, n);
    bool conv = false;
    double rel = 1.0;
    fgmres(P, ops, g, lam, P.rwork, o.tol, o.restart, maxit, st, S, conv, rel, true, o);
    S.refinements = 1;
    S.converged = conv ? 1 : 0;
    S.rel_res = rel;
    S.t_total = now() - t_start;
    return conv ? TSFDE_OK : TSFDE_ENOCONV;
}

// ---------------------------------------------------------------------------
// Spectral tools (§6.1.1, §6.2: the 2-norm condition numbers of A and P^{-1} A)
// ---------------------------------------------------------------------------
static double norm2(Problem& P, const double* x, hipStream_t st) { return std::sqrt(dev_dot(P, x, x, P.ntot, st)); }

// The largest eigenvalue of a symmetric positive operator op by Lanczos with full reorthogonalisation
// (Arnoldi with classical Gram-Schmidt twice on a symmetric operator; Q holds kmax + 1 vectors): the
// largest Ritz value of the k x k matrix after each step, stopping when it changes by less than 1e-12
// relative in two consecutive steps, at kmax steps, or on an exact breakdown.  *steps: steps taken.
static double lanczos_max(Problem& P, const std::function<tsfde_status(const double*, double*)>& op, double* Q,
                          int kmax, unsigned long long seed, int* steps, tsfde_status& rc, hipStream_t st) {
    const long long n = P.ntot;
    if (!P.arn_part) dev_alloc(P, P.arn_part, kArnBlocks * kArnMaxK);
    if (!P.arn_h) dev_alloc(P, P.arn_h, (2 * (kMaxRestart + 2) + 1));
    const int hs = kmax + 2;
    std::vector<double> H((size_t)(kmax + 1) * kmax, 0.0), hhost(2 * hs + 1), A, re, im;
    launch_hash_fill(Q, n, seed, st);
    launch_axpby(1.0 / std::sqrt(dev_dot(P, Q, Q, n, st)), Q, 0.0, Q, Q, n, st);
    double lam = 0.0, prev = -1.0;
    int calm = 0, k = 0;
    rc = TSFDE_OK;
    for (; k < kmax; ++k) {
        double* w = Q + (size_t)(k + 1) * n;
        rc = op(Q + (size_t)k * n, w);
        if (rc != TSFDE_OK) break;
        cgs2(Q, n, k + 1, w, P.arn_part, kArnBlocks, P.arn_h, P.arn_h + hs, P.arn_h + 2 * hs, st);
        TSFDE_HIP(hipMemcpyAsync(hhost.data(), P.arn_h, sizeof(double) * (2 * hs + 1), hipMemcpyDeviceToHost, st));
        TSFDE_HIP(hipStreamSynchronize(st));
        for (int i = 0; i <= k; ++i) H[(size_t)i * kmax + k] = hhost[i] + hhost[hs + i];
        const double hn = std::sqrt(hhost[2 * hs]);
        H[(size_t)(k + 1) * kmax + k] = hn;
        // Ritz values of the leading (k+1) x (k+1) block
        const int m = k + 1;
        A.assign((size_t)m * m, 0.0);
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < m; ++c) A[(size_t)r * m + c] = H[(size_t)r * kmax + c];
        if (hessenberg_eigenvalues(A, m, re, im)) {
            lam = 0.0;
            for (int r = 0; r < m; ++r) lam = std::max(lam, re[r]);
        }
        calm = (prev > 0.0 && std::fabs(lam - prev) <= 1e-12 * lam) ? calm + 1 : 0;
        prev = lam;
        if (calm >= 2 || !(hn > 1e-14 * lam)) { ++k; break; }
        launch_axpby(1.0 / hn, w, 0.0, w, w, n, st);
    }
    *steps = k;
    return lam;
}

// sigma_max and sigma_min of M = A or P^{-1} A: sigma_max^2 the largest eigenvalue of M^T M and
// 1 / sigma_min^2 that of (M^T M)^{-1} = M^{-1} M^{-T}, both by Lanczos.  P^{-1} and P^{-T} are applied
// with o.inner_tol (fixed linear operators: a tight tolerance); M^{-1} = A^{-1} P and M^{-T} = P^T A^{-T}
// by FGMRES with A and A^T to o.tol.  used[0], used[1]: the Lanczos steps.
static tsfde_status singular_values_impl(Problem& P, int precond, int kmax, double& smax, double& smin, int* used,
                                         const Opts& o, hipStream_t st) {
    const long long n = P.ntot;
    const size_t nvec = (size_t)kmax + 3;
    if (P.spec_vecs < nvec) {
        if (P.spec_work) {
            (void)hipFree(P.spec_work);
            P.bytes -= sizeof(double) * P.spec_vecs * (size_t)n;
            P.spec_work = nullptr;
            P.spec_vecs = 0;
        }
        dev_alloc(P, P.spec_work, nvec * (size_t)n);
        P.spec_vecs = nvec;
    }
    double* w = P.spec_work;       // operator scratch
    double* t = w + n;             // operator scratch
    double* Q = w + 2 * n;         // Lanczos vectors (kmax + 1)
    Opts so = o;
    so.precision = TSFDE_FP64;
    so.use_precond = 1;
    so.maxit = o.maxit > 0 ? o.maxit : 1000;
    tsfde_stats S{};
    auto MtM = [&](const double* in, double* out) -> tsfde_status {  // out = M^T M in
        if (precond) {
            apply_A_impl<double>(P, in, w, st);
            pinv_impl<double>(P, w, t, so, st, true);
            ptinv_launch(P, t, w, so, st);
            apply_AT_impl(P, w, out, st);
        } else {
            apply_A_impl<double>(P, in, w, st);
            apply_AT_impl(P, w, out, st);
        }
        return TSFDE_OK;
    };
    auto MtMinv = [&](const double* in, double* out) -> tsfde_status {  // out = M^{-1} M^{-T} in
        // t = M^{-T} in = P^T A^{-T} in
        launch_fill(w, n, 0.0, st);
        tsfde_status rc = adjoint_impl(P, in, w, so, S, st);
        if (rc != TSFDE_OK) return rc;
        if (precond) {
            apply_AT_impl(P, w, t, st);
            launch_coupling(P, w, t, true, st);
        } else {
            launch_copy<double>(w, t, n, st);
        }
        // out = M^{-1} t = A^{-1} (P t)
        const double* b = t;
        if (precond) {
            apply_A_impl<double>(P, t, w, st);
            launch_coupling(P, t, w, false, st);
            b = w;
        }
        launch_fill(out, n, 0.0, st);
        return solve(P, b, out, so, S, st);
    };
    tsfde_status rc = TSFDE_OK;
    smax = std::sqrt(lanczos_max(P, MtM, Q, kmax, 0x7a3f11ull, &used[0], rc, st));
    if (rc != TSFDE_OK) return rc;
    smin = 1.0 / std::sqrt(lanczos_max(P, MtMinv, Q, kmax, 0x51c9e2ull, &used[1], rc, st));
    if (rc != TSFDE_OK) return rc;
    TSFDE_HIP(hipStreamSynchronize(st));
    return TSFDE_OK;
}

// Morozov's discrepancy of a source f (device): || v^(M)(f) - mu_eps ||_2 with v the direct problem's
// solution for f (§6.1), the first M steps of the forward substitution
static double discrepancy_impl(Problem& P, const double* f, const Opts& o, hipStream_t st) {
    if (!P.fwd_work) dev_alloc(P, P.fwd_work, 2 * (size_t)P.ntot);
    double* zh = P.fwd_work;
    double* y = P.fwd_work + P.ntot;
    Opts fo = o;
    fo.block_solver = TSFDE_BLOCK_CG;  // the direct problem is solved, not preconditioned
    launch_build_zhat(P, f, zh, st);
    pinv_impl<double>(P, zh, y, fo, st, false);
    launch_axpby(1.0, y + (size_t)(P.M - 1) * P.Nd, -1.0, P.d_mu, zh, P.Nd, st);
    return std::sqrt(dev_dot(P, zh, zh, P.Nd, st));
}

}  // namespace tsfde

// ===========================================================================
// C ABI
// ===========================================================================
using namespace tsfde;

struct tsfde_problem {
    Problem* p;
};

#define TSFDE_GUARD(name, body)                                                           \
    try {                                                                                 \
        body                                                                              \
    } catch (const HipError& e) {                                                         \
        set_error("%s: %s failed: %s", name, e.where.c_str(), hipGetErrorString(e.code)); \
        return e.code == hipErrorOutOfMemory ? TSFDE_ENOMEM : TSFDE_EDEVICE;              \
    } catch (const CapError& e) {                                                         \
        set_error("%s: %s", name, e.msg.c_str());                                         \
        return TSFDE_ENOMEM;                                                              \
    } catch (const std::bad_alloc&) {                                                     \
        set_error("%s: host allocation failed", name);                                    \
        return TSFDE_ENOMEM;                                                              \
    }

static bool overlap(const void* a, const void* b, size_t bytes) {
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + bytes && y < x + bytes;
}

// Builds z, solves from x0 = 0 into work (or the problem's buffer) and copies f~ out; synchronises st.
static tsfde_status recover_impl(Problem& P, double* f_out, double* work, const Opts& o, tsfde_stats& S,
                                 hipStream_t st) {
    tsfde_status rc = TSFDE_OK;
    TSFDE_GUARD("recover_f", {
        double* x = work;
        if (!x) {
            if (!P.xbuf) dev_alloc(P, P.xbuf, P.ntot);
            x = P.xbuf;
        }
        launch_fill(x, P.ntot, 0.0, st);
        launch_build_z(P, P.z_rhs, st);
        rc = solve(P, P.z_rhs, x, o, S, st);
        launch_copy<double>(x + (size_t)P.M * P.Nd, f_out, P.Nd, st);
        TSFDE_HIP(hipStreamSynchronize(st));
    })
    if (rc == TSFDE_ENOCONV) set_error("recover_f: tolerance not reached (rel. residual %.3e)", S.rel_res);
    return rc;
}

// Block FGMRES on p right-hand sides (FP64, or PREC_F32: the preconditioner in FP32); B and X hold p
// vectors of n_tot, X the initial guesses.  rel_out (host, p) gets each column's relative residual.
static tsfde_status solve_block(Problem& P, int p, const double* B, double* X, double* rel_out, const Opts& o,
                                tsfde_stats& S, hipStream_t st) {
    const long long n = P.ntot;
    const int maxit = o.maxit > 0 ? o.maxit : (int)std::min<long long>(n, 1000);
    const double t_start = now();
    P.res_hist.clear();
    struct History {
        Problem& P;
        tsfde_stats& S;
        ~History() {
            S.history_len = (int)P.res_hist.size();
            S.history = P.res_hist.data();
        }
    } hist{P, S};
    SolveOps ops;
    ops.A = [&](const double* v, double* out) { apply_A_impl<double>(P, v, out, st); };
    Opts o32 = o;
    o32.inner_tol = std::max(o.inner_tol, kInnerTolF32);
    Dev<float>& F = P.f32;
    if (o.precision == TSFDE_PREC_F32 && !F.vecA) {
        dev_alloc(P, F.vecA, n);
        dev_alloc(P, F.vecB, n);
    }
    ops.M = [&](const double* v, double* out) -> long long {
        if (!o.use_precond) { launch_copy<double>(v, out, n, st); return 0; }
        if (o.precision == TSFDE_FP64) return pinv_impl<double>(P, v, out, o, st, true);
        launch_d2f(v, F.vecA, n, st);
        const long long it = pinv_impl<float>(P, F.vecA, F.vecB, o32, st, true);
        launch_f2d(F.vecB, out, n, st);
        return it;
    };
    std::vector<double> rel;
    bool conv = false;
    block_fgmres(P, ops, p, B, X, o.tol, o.restart, maxit, st, S, rel, conv, o);
    double worst = 0.0;
    for (int c = 0; c < p; ++c) worst = std::max(worst, rel[c]);
    if (rel_out) std::copy(rel.begin(), rel.end(), rel_out);
    S.refinements = 1;
    S.converged = conv ? 1 : 0;
    S.rel_res = worst;
    TSFDE_HIP(hipStreamSynchronize(st));
    S.t_total = now() - t_start;
    return conv ? TSFDE_OK : TSFDE_ENOCONV;
}

static bool check_block(const Problem& P, int nrhs, const Opts& o, const char* name) {
    if (nrhs < 1 || nrhs > kBlockMaxCols) {
        set_error("%s: nrhs must be in [1, %d]", name, kBlockMaxCols);
        return false;
    }
    if ((long long)o.restart * nrhs > kBlockMaxBasis) {
        set_error("%s: restart * nrhs must be <= %d", name, kBlockMaxBasis);
        return false;
    }
    if (o.precision == TSFDE_MIXED) {
        set_error("%s: precision MIXED is not available for blocks (FP64 or PREC_F32)", name);
        return false;
    }
    (void)P;
    return true;
}

// The vector-Jacobian product of f~ (see tsfde_recover_f_vjp); synchronises st.
static tsfde_status vjp_impl(Problem& P, const double* y, const double* gf, double* grad_mu, double* grad_alpha,
                             double* grad_gamma2, const Opts& o, tsfde_stats& S, hipStream_t st) {
    const long long n = P.ntot, Nd = P.Nd, last = (long long)P.M * P.Nd;
    tsfde_status rc = TSFDE_OK;
    TSFDE_GUARD("recover_f_vjp", {
        // g = [0; gf], lam, then v = [0; y^(M)] and A v (problem-owned, allocated on first use)
        if (!P.vjp_work) dev_alloc(P, P.vjp_work, 3 * (size_t)n);
        double* w = P.vjp_work;
        double* g = w;
        double* lam = w + n;
        double* v = w + 2 * n;
        launch_fill(g, n, 0.0, st);
        launch_copy<double>(gf, g + last, Nd, st);
        launch_fill(lam, n, 0.0, st);
        {
            rc = adjoint_impl(P, g, lam, o, S, st);
            if (grad_mu) launch_copy<double>(lam + last, grad_mu, Nd, st);
            if (grad_gamma2) {
                // v = (c_t B y^(s), c_f B y^(M)): the matvec's B kernels with unit gamma2 into a zero
                // vector, the last row adding the (zero) first slice of g instead of y^(M-1)
                Dev<double> Dn = P.f64;
                Dn.gamma2 = nullptr;
                launch_fill(v, n, 0.0, st);
                if (!launch_toeplitz2d_matvec<double>(P, Dn, y, v, st, g))
                    launch_toeplitz_matvec<double>(P, Dn, y, v, st, g);
                launch_gamma2_grad(P, lam, v, grad_gamma2, st);
            }
            if (grad_alpha) {
                // dA/dalpha y = (1/alpha) (A [0; y^(M)])^(M): only c_f = alpha/h^omega depends on alpha
                launch_fill(v, n, 0.0, st);
                launch_copy<double>(y + last, v + last, Nd, st);
                apply_A_impl<double>(P, v, g, st);
                *grad_alpha = -dev_dot(P, lam + last, g + last, Nd, st) / P.alpha;
            }
            TSFDE_HIP(hipStreamSynchronize(st));
        }
    })
    if (rc == TSFDE_ENOCONV) set_error("recover_f_vjp: adjoint tolerance not reached (rel. residual %.3e)", S.rel_res);
    return rc;
}

// Several problems solved in lockstep with their P^{-1} applications in shared persistent launches
// (pinv_multi_run): each Arnoldi step applies P^{-1} to the current basis vector of every unfinished
// problem in one set of launches (one launch per round of kHB time steps and kernel form), then runs
// each problem's matvec and Gram-Schmidt on the stream and its Givens rotations on the host.  FGMRES
// is the single-problem one otherwise: restart cycles per problem, the true residual at every
// (re)start, x0 = 0, f~ = the last block.  FP64, CG blocks, directions kept.
static tsfde_status recover_multi_impl(const std::vector<Problem*>& probs, double* const* f_out, const Opts& o,
                                       tsfde_stats* stats, hipStream_t st) {
    struct Slot {
        Problem* P = nullptr;
        tsfde_stats S{};
        bool done = false, conv = false;
        int its = 0, j = 0, maxit = 0;
        double bnorm = 0.0, t0 = 0.0;
        std::vector<double> Hc, cs, sn, g, yk, hh;
    };
    const int m = o.restart, hs = m + 2;
    const int nblk = kArnBlocks;
    const int extrap = env_int("TSFDE_EXTRAP", o.warm_start);
    std::vector<Slot> sl(probs.size());
    auto vec = [](Problem& P, int k) { return P.V + (size_t)k * P.ntot; };
    // r = b - A x and the true relative residual; a new cycle from it unless converged or out of steps
    auto start_cycle = [&](Slot& q) {
        Problem& P = *q.P;
        const long long n = P.ntot;
        const double t0 = now();
        apply_A_impl<double>(P, P.xbuf, P.rwork, st);
        launch_axpby(1.0, P.z_rhs, -1.0, P.rwork, P.rwork, n, st);
        const double beta = std::sqrt(dev_dot(P, P.rwork, P.rwork, n, st));
        q.S.t_matvec += now() - t0;
        const double rel = q.bnorm > 0.0 ? beta / q.bnorm : 0.0;
        P.res_hist.push_back(rel);
        q.S.rel_res = rel;
        if (rel <= o.tol) { q.done = true; q.conv = true; return; }
        if (q.its >= q.maxit || !(beta > 0.0)) { q.done = true; return; }
        launch_axpby(1.0 / beta, P.rwork, 0.0, P.rwork, P.V, n, st);
        std::fill(q.g.begin(), q.g.end(), 0.0);
        q.g[0] = beta;
        q.j = 0;
    };
    for (size_t i = 0; i < probs.size(); ++i) {
        Slot& q = sl[i];
        q.P = probs[i];
        Problem& P = *q.P;
        const long long n = P.ntot;
        q.t0 = now();
        q.maxit = o.maxit > 0 ? o.maxit : (int)std::min<long long>(n, 1000);
        P.res_hist.clear();
        if (ensure_basis(P, m, o)) throw CapError{"multi solve: the directions z_j do not fit (recomputing them is not offered here)"};
        if (!P.arn_part) dev_alloc(P, P.arn_part, kArnBlocks * kArnMaxK);
        if (!P.arn_h) dev_alloc(P, P.arn_h, (2 * (kMaxRestart + 2) + 1));
        if (!P.xbuf) dev_alloc(P, P.xbuf, n);
        if (!P.rwork) dev_alloc(P, P.rwork, n);
        q.Hc.assign((size_t)(m + 1) * m, 0.0);
        q.cs.assign(m, 0.0);
        q.sn.assign(m, 0.0);
        q.g.assign(m + 1, 0.0);
        q.yk.assign(m, 0.0);
        q.hh.assign(2 * hs + 1, 0.0);
        launch_fill(P.xbuf, n, 0.0, st);
        launch_build_z(P, P.z_rhs, st);
        q.bnorm = std::sqrt(dev_dot(P, P.z_rhs, P.z_rhs, n, st));
        if (!(q.bnorm > 0.0)) { q.done = true; q.conv = true; q.S.rel_res = 0.0; continue; }
        start_cycle(q);
    }
    std::vector<PinvMultiJob> jobs;
    std::vector<int> who;
    while (true) {
        jobs.clear();
        who.clear();
        for (size_t i = 0; i < sl.size(); ++i)
            if (!sl[i].done) {
                Problem& P = *sl[i].P;
                jobs.push_back(PinvMultiJob{&P, vec(P, sl[i].j), P.Z + (size_t)sl[i].j * P.ntot, 0});
                who.push_back((int)i);
            }
        if (jobs.empty()) break;
        double t0 = now();
        if (o.use_precond) {
            pinv_multi_run(jobs, o.inner_tol, o.inner_maxit, extrap, st);  // synchronises st
        } else {
            for (auto& jb : jobs) launch_copy<double>(jb.z, jb.y, jb.P->ntot, st);
        }
        const double tp = now() - t0;
        t0 = now();
        for (size_t k = 0; k < who.size(); ++k) {
            Slot& q = sl[who[k]];
            Problem& P = *q.P;
            q.S.t_precond += tp;
            q.S.inner_iters += jobs[k].iters;
            double* w = vec(P, q.j + 1);
            apply_A_impl<double>(P, P.Z + (size_t)q.j * P.ntot, w, st);
            cgs2(P.V, P.ntot, q.j + 1, w, P.arn_part, nblk, P.arn_h, P.arn_h + hs, P.arn_h + 2 * hs, st);
            TSFDE_HIP(hipMemcpyAsync(q.hh.data(), P.arn_h, sizeof(double) * (2 * hs + 1), hipMemcpyDeviceToHost, st));
        }
        TSFDE_HIP(hipStreamSynchronize(st));
        const double tm = now() - t0;
        for (int i : who) {
            Slot& q = sl[i];
            Problem& P = *q.P;
            q.S.t_ortho += tm / (double)who.size();
            const int j = q.j;
            const double hn = std::sqrt(std::max(0.0, q.hh[2 * hs]));
            for (int r = 0; r <= j; ++r) q.Hc[(size_t)r * m + j] = q.hh[r] + q.hh[hs + r];
            q.Hc[(size_t)(j + 1) * m + j] = hn;
            for (int r = 0; r < j; ++r) {
                const double a = q.Hc[(size_t)r * m + j], bq = q.Hc[(size_t)(r + 1) * m + j];
                q.Hc[(size_t)r * m + j] = q.cs[r] * a + q.sn[r] * bq;
                q.Hc[(size_t)(r + 1) * m + j] = -q.sn[r] * a + q.cs[r] * bq;
            }
            const double a = q.Hc[(size_t)j * m + j], bq = q.Hc[(size_t)(j + 1) * m + j];
            const double rr = std::hypot(a, bq);
            q.cs[j] = rr > 0.0 ? a / rr : 1.0;
            q.sn[j] = rr > 0.0 ? bq / rr : 0.0;
            q.Hc[(size_t)j * m + j] = rr;
            q.Hc[(size_t)(j + 1) * m + j] = 0.0;
            q.g[j + 1] = -q.sn[j] * q.g[j];
            q.g[j] = q.cs[j] * q.g[j];
            ++q.its;
            ++q.S.iters;
            P.res_hist.push_back(std::fabs(q.g[j + 1]) / q.bnorm);
            const bool end = std::fabs(q.g[j + 1]) <= o.tol * q.bnorm || j + 1 == m || q.its >= q.maxit || hn == 0.0;
            if (!end) {
                launch_axpby(1.0 / hn, vec(P, j + 1), 0.0, vec(P, j + 1), vec(P, j + 1), P.ntot, st);
                q.j = j + 1;
                continue;
            }
            const int k = j + 1;
            for (int r = k - 1; r >= 0; --r) {
                double acc = q.g[r];
                for (int l = r + 1; l < k; ++l) acc -= q.Hc[(size_t)r * m + l] * q.yk[l];
                q.yk[r] = q.Hc[(size_t)r * m + r] != 0.0 ? acc / q.Hc[(size_t)r * m + r] : 0.0;
            }
            TSFDE_HIP(hipMemcpyAsync(P.arn_h, q.yk.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
            launch_gemv_add(P.Z, P.ntot, k, P.arn_h, P.xbuf, st);
            TSFDE_HIP(hipStreamSynchronize(st));
            ++q.S.restarts;
            start_cycle(q);
        }
    }
    tsfde_status rc = TSFDE_OK;
    for (size_t i = 0; i < sl.size(); ++i) {
        Slot& q = sl[i];
        Problem& P = *q.P;
        launch_copy<double>(P.xbuf + (size_t)P.M * P.Nd, f_out[i], P.Nd, st);
        q.S.converged = q.conv ? 1 : 0;
        q.S.refinements = 1;
        q.S.t_total = now() - q.t0;
        q.S.history_len = (int)P.res_hist.size();
        q.S.history = P.res_hist.data();
        if (stats) stats[i] = q.S;
        if (!q.conv && rc == TSFDE_OK) rc = TSFDE_ENOCONV;
    }
    TSFDE_HIP(hipStreamSynchronize(st));
    return rc;
}

// Runs fn(i, problem i, its stats, a stream) for every problem of a batch, up to max_inflight at once,
// each worker thread on a non-blocking stream of its own, largest problems first; the persistent
// grids of the workers are limited so that that many fit together, and every persistent grid of the
// process holds its share of the device's CU slots while it runs (residency.hpp).  Checks the batch
// and returns the first device error by index, else TSFDE_ENOCONV if any problem missed its tolerance.
template <typename F>
static tsfde_status run_batch(const char* name, tsfde_problem* const* probs, int count, const Opts& o,
                              tsfde_stats* stats, int max_inflight, void* stream, F&& fn) {
    if (max_inflight < 1 || max_inflight > kMaxInflight) {
        set_error("%s: max_inflight must be in [1, %d]", name, kMaxInflight);
        return TSFDE_EINVAL;
    }
    for (int i = 0; i < count; ++i) {
        if (!probs[i]) {
            set_error("%s: problem %d is NULL", name, i);
            return TSFDE_EINVAL;
        }
        for (int j = 0; j < i; ++j)
            if (probs[j] == probs[i]) {
                set_error("%s: problem %d appears twice (entries %d and %d)", name, i, j, i);
                return TSFDE_EINVAL;
            }
        if (!block_solver_supported(*probs[i]->p, o)) return TSFDE_ENOTIMPL;
    }
    if (count == 0) return TSFDE_OK;
    int dev = 0;
    TSFDE_GUARD(name, {
        TSFDE_HIP(hipGetDevice(&dev));
        TSFDE_HIP(hipStreamSynchronize((hipStream_t)stream));
    })
    std::vector<tsfde_status> rcs(count, TSFDE_OK);
    std::vector<std::string> msgs(count);
    std::vector<tsfde_stats> S(count, tsfde_stats{});
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return probs[x]->p->ntot > probs[y]->p->ntot; });
    std::atomic<int> next{0};
    auto worker = [&]() {
        hipStream_t st = nullptr;
        hipError_t e = hipSetDevice(dev);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        set_shared_launch(true);
        for (int t; (t = next.fetch_add(1)) < count;) {
            const int i = order[t];
            if (e != hipSuccess) {
                rcs[i] = TSFDE_EDEVICE;
                msgs[i] = std::string("stream creation failed: ") + hipGetErrorString(e);
                continue;
            }
            rcs[i] = fn(i, *probs[i]->p, S[i], st);
            if (rcs[i] != TSFDE_OK) msgs[i] = last_error();
        }
        set_shared_launch(false);
        if (st) (void)hipStreamDestroy(st);
    };
    std::vector<std::thread> th;
    try {
        for (int t = 1; t < std::min(max_inflight, count); ++t) th.emplace_back(worker);
    } catch (const std::system_error&) {
        // fewer workers: the calling thread and those started take every problem
    }
    worker();
    for (auto& t : th) t.join();
    if (stats)
        for (int i = 0; i < count; ++i) stats[i] = S[i];
    for (int i = 0; i < count; ++i)
        if (rcs[i] != TSFDE_OK && rcs[i] != TSFDE_ENOCONV) {
            set_error("%s: problem %d: %s", name, i, msgs[i].c_str());
            return rcs[i];
        }
    for (int i = 0; i < count; ++i)
        if (rcs[i] == TSFDE_ENOCONV) {
            set_error("%s: problem %d: %s", name, i, msgs[i].c_str());
            return TSFDE_ENOCONV;
        }
    return TSFDE_OK;
}

extern "C" {

void tsfde_default_opts(tsfde_opts* o) {
    if (!o) return;
    o->restart = 50;
    o->maxit = 0;
    o->tol = 1e-10;
    o->precision = TSFDE_FP64;
    o->block_solver = TSFDE_BLOCK_CG;
    o->warm_start = TSFDE_WARM_LINEAR;
    o->use_precond = 1;
    o->inner_tol = 1e-12;
    o->inner_maxit = 200;
    o->refine_tol = 1e-5;
    o->max_refine = 30;
    o->max_device_bytes = 0;
    o->recompute_z = 0;
    o->graph = 0;
}

tsfde_status tsfde_create_problem_ex(int d, int N, int M, double T, double beta, double omega, double alpha,
                                     const double* gamma1, const double* gamma2, const double* q, const double* rho,
                                     const double* mu, double length, const double* stencil, tsfde_problem** out) {
    if (!out) {
        set_error("create_problem: out is NULL");
        return TSFDE_EINVAL;
    }
    *out = nullptr;
    Problem* P = nullptr;
    tsfde_status st = create(d, N, M, T, beta, omega, alpha, gamma1, gamma2, q, rho, mu, length, stencil, &P);
    if (st != TSFDE_OK) return st;
    *out = new tsfde_problem{P};
    return TSFDE_OK;
}

tsfde_status tsfde_create_problem(int d, int N, int M, double T, double beta, double omega, double alpha,
                                  const double* gamma1, const double* gamma2, const double* q, const double* rho,
                                  const double* mu, tsfde_problem** out) {
    return tsfde_create_problem_ex(d, N, M, T, beta, omega, alpha, gamma1, gamma2, q, rho, mu, 1.0, nullptr, out);
}

tsfde_status tsfde_set_mu(tsfde_problem* prob, const double* mu) {
    if (!prob) { set_error("set_mu: NULL problem"); return TSFDE_EINVAL; }
    return set_mu(prob->p, mu);
}

tsfde_status tsfde_set_gamma2(tsfde_problem* prob, const double* gamma2) {
    if (!prob) { set_error("set_gamma2: NULL problem"); return TSFDE_EINVAL; }
    return set_gamma2(prob->p, gamma2);
}

tsfde_status tsfde_set_alpha(tsfde_problem* prob, double alpha) {
    if (!prob) { set_error("set_alpha: NULL problem"); return TSFDE_EINVAL; }
    if (!(alpha > 0.0) || !std::isfinite(alpha)) { set_error("set_alpha: need alpha > 0"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    P.alpha = alpha;  // only the final-condition block's coefficient depends on alpha
    P.cf = alpha / std::pow(P.h, P.omega);
    return TSFDE_OK;
}

void tsfde_destroy_problem(tsfde_problem* prob) {
    if (!prob) return;
    free_problem(prob->p);
    delete prob;
}

size_t tsfde_vector_length(const tsfde_problem* prob) { return prob ? (size_t)prob->p->ntot : 0; }

size_t tsfde_device_bytes(const tsfde_problem* prob) { return prob ? prob->p->bytes : 0; }

tsfde_status tsfde_problem_scalars(const tsfde_problem* prob, double out[6]) {
    if (!prob || !out) { set_error("problem_scalars: NULL argument"); return TSFDE_EINVAL; }
    const Problem& P = *prob->p;
    out[0] = P.h;
    out[1] = P.dt;
    out[2] = P.eta;
    out[3] = P.ct;
    out[4] = P.cf;
    out[5] = P.L;
    return TSFDE_OK;
}

tsfde_status tsfde_get_stencil(const tsfde_problem* prob, double* out) {
    if (!prob || !out) { set_error("get_stencil: NULL argument"); return TSFDE_EINVAL; }
    std::copy(prob->p->stencil.begin(), prob->p->stencil.end(), out);
    return TSFDE_OK;
}

tsfde_status tsfde_compute_stencil(int d, int N, double omega, double* out) {
    return compute_stencil(d, N, omega, out);
}

tsfde_status tsfde_apply_A(tsfde_problem* prob, const double* y, double* z, void* stream) {
    if (!prob || !y || !z) { set_error("apply_A: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    if (overlap(y, z, sizeof(double) * P.ntot)) { set_error("apply_A: y and z overlap"); return TSFDE_EINVAL; }
    TSFDE_GUARD("apply_A", apply_A_impl<double>(P, y, z, (hipStream_t)stream);)
    return TSFDE_OK;
}

tsfde_status tsfde_apply_A_f32(tsfde_problem* prob, const float* y, float* z, void* stream) {
    if (!prob || !y || !z) { set_error("apply_A_f32: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    if (overlap(y, z, sizeof(float) * P.ntot)) { set_error("apply_A_f32: y and z overlap"); return TSFDE_EINVAL; }
    TSFDE_GUARD("apply_A_f32", apply_A_impl<float>(P, y, z, (hipStream_t)stream);)
    return TSFDE_OK;
}

tsfde_status tsfde_apply_P_inv(tsfde_problem* prob, const double* z, double* y, const tsfde_opts* opts, void* stream) {
    if (!prob || !y || !z) { set_error("apply_P_inv: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    if (overlap(y, z, sizeof(double) * P.ntot)) { set_error("apply_P_inv: y and z overlap"); return TSFDE_EINVAL; }
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    if (!block_solver_supported(P, o)) return TSFDE_ENOTIMPL;
    TSFDE_GUARD("apply_P_inv", pinv_impl<double>(P, z, y, o, (hipStream_t)stream, true);)
    return TSFDE_OK;
}

tsfde_status tsfde_apply_P_inv_noalloc(tsfde_problem* prob, const double* z, double* y, const tsfde_opts* opts,
                                       void* stream) {
    if (!prob || !y || !z) { set_error("apply_P_inv_noalloc: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    if (overlap(y, z, sizeof(double) * P.ntot)) { set_error("apply_P_inv_noalloc: y and z overlap"); return TSFDE_EINVAL; }
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    if (o.block_solver == TSFDE_BLOCK_STRANG) {
        set_error("apply_P_inv_noalloc: TSFDE_BLOCK_STRANG builds device tables on first use; use tsfde_apply_P_inv");
        return TSFDE_ENOTIMPL;
    }
    if (!persistent_supported(P)) {
        set_error("apply_P_inv_noalloc: this shape has no persistent forward-substitution kernel (L = %d)", P.L);
        return TSFDE_ENOTIMPL;
    }
    if (o.block_solver == TSFDE_BLOCK_TAU && !tau_persistent(P)) {
        set_error("apply_P_inv_noalloc: TSFDE_BLOCK_TAU on this shape uses the dense sine passes, whose tables are "
                  "built on first use; use tsfde_apply_P_inv");
        return TSFDE_ENOTIMPL;
    }
    if (!block_solver_supported(P, o)) return TSFDE_ENOTIMPL;
    const size_t need = pinv_noalloc_bytes(P);
    if (need > kNoAllocScratchBytes) {
        set_error("apply_P_inv_noalloc: the problem needs %zu bytes of scratch, the static scratch holds %zu", need,
                  kNoAllocScratchBytes);
        return TSFDE_ENOMEM;
    }
    // calls on one device share its scratch: they are serialised (each call ends synchronised)
    static std::mutex mx[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        set_error("apply_P_inv_noalloc: no usable current device");
        return TSFDE_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(mx[dev]);
    set_persistent_blocks(env_int("TSFDE_PINV_BLOCKS", -1));
    set_persistent_fixed_length(env_int("TSFDE_PINV_FIXED", 1) != 0);
    TSFDE_GUARD("apply_P_inv_noalloc",
                pinv_persistent_run_noalloc(P, z, y, o.inner_tol, o.inner_maxit, env_int("TSFDE_EXTRAP", o.warm_start),
                                            o.block_solver == TSFDE_BLOCK_TAU ? 1 : 0, (hipStream_t)stream);)
    return TSFDE_OK;
}

tsfde_status tsfde_apply_P_inv_f32(tsfde_problem* prob, const float* z, float* y, const tsfde_opts* opts,
                                   void* stream) {
    if (!prob || !y || !z) { set_error("apply_P_inv_f32: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    if (overlap(y, z, sizeof(float) * P.ntot)) { set_error("apply_P_inv_f32: y and z overlap"); return TSFDE_EINVAL; }
    Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    if (!block_solver_supported(P, o)) return TSFDE_ENOTIMPL;
    o.inner_tol = std::max(o.inner_tol, kInnerTolF32);
    TSFDE_GUARD("apply_P_inv_f32", pinv_impl<float>(P, z, y, o, (hipStream_t)stream, true);)
    return TSFDE_OK;
}

tsfde_status tsfde_gmres_solve(tsfde_problem* prob, const double* b, double* x, const tsfde_opts* opts,
                               tsfde_stats* stats, void* stream) {
    if (!prob || !x) { set_error("gmres_solve: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    if (b && overlap(b, x, sizeof(double) * P.ntot)) { set_error("gmres_solve: b and x overlap"); return TSFDE_EINVAL; }
    if (!block_solver_supported(P, o)) return TSFDE_ENOTIMPL;
    tsfde_stats S{};
    tsfde_status rc = TSFDE_OK;
    hipStream_t st = (hipStream_t)stream;
    TSFDE_GUARD("gmres_solve", {
        if (!b) {
            launch_build_z(P, P.z_rhs, st);
            b = P.z_rhs;
        }
        rc = solve(P, b, x, o, S, st);
    })
    if (stats) *stats = S;
    if (rc == TSFDE_ENOCONV) set_error("gmres_solve: tolerance not reached (rel. residual %.3e)", S.rel_res);
    return rc;
}

tsfde_status tsfde_recover_f(tsfde_problem* prob, double* f_out, double* work, const tsfde_opts* opts,
                             tsfde_stats* stats, void* stream) {
    if (!prob || !f_out) { set_error("recover_f: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    if (!block_solver_supported(P, o)) return TSFDE_ENOTIMPL;
    tsfde_stats S{};
    const tsfde_status rc = recover_impl(P, f_out, work, o, S, (hipStream_t)stream);
    if (stats) *stats = S;
    return rc;
}

tsfde_status tsfde_recover_f_batch(tsfde_problem* const* probs, int count, double* const* f_out,
                                   const tsfde_opts* opts, tsfde_stats* stats, int max_inflight, void* stream) {
    if (count < 0 || (count > 0 && (!probs || !f_out))) {
        set_error("recover_f_batch: count < 0 or NULL arrays");
        return TSFDE_EINVAL;
    }
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!f_out[i]) {
            set_error("recover_f_batch: output %d is NULL", i);
            return TSFDE_EINVAL;
        }
    return run_batch("recover_f_batch", probs, count, o, stats, max_inflight, stream,
                     [&](int i, Problem& P, tsfde_stats& S, hipStream_t st) {
                         return recover_impl(P, f_out[i], nullptr, o, S, st);
                     });
}

tsfde_status tsfde_recover_f_vjp_batch(tsfde_problem* const* probs, int count, const double* const* ys,
                                       const double* const* gfs, double* const* grad_mu, double* grad_alpha,
                                       double* const* grad_gamma2, const tsfde_opts* opts, tsfde_stats* stats,
                                       int max_inflight, void* stream) {
    if (count < 0 || (count > 0 && (!probs || !gfs))) {
        set_error("recover_f_vjp_batch: count < 0 or NULL arrays");
        return TSFDE_EINVAL;
    }
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (!gfs[i]) {
            set_error("recover_f_vjp_batch: gf %d is NULL", i);
            return TSFDE_EINVAL;
        }
        if (probs && probs[i] && !(ys && ys[i]) && !probs[i]->p->xbuf) {
            set_error("recover_f_vjp_batch: problem %d has no solution (no ys and no earlier recover_f)", i);
            return TSFDE_EINVAL;
        }
    }
    return run_batch("recover_f_vjp_batch", probs, count, o, stats, max_inflight, stream,
                     [&](int i, Problem& P, tsfde_stats& S, hipStream_t st) {
                         return vjp_impl(P, (ys && ys[i]) ? ys[i] : P.xbuf, gfs[i], grad_mu ? grad_mu[i] : nullptr,
                                         grad_alpha ? grad_alpha + i : nullptr,
                                         grad_gamma2 ? grad_gamma2[i] : nullptr, o, S, st);
                     });
}

tsfde_status tsfde_gmres_solve_block(tsfde_problem* prob, int nrhs, const double* B, double* X, double* rel_res,
                                     const tsfde_opts* opts, tsfde_stats* stats, void* stream) {
    if (!prob || !B || !X) { set_error("gmres_solve_block: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    if (!check_block(P, nrhs, o, "gmres_solve_block")) return TSFDE_ENOTIMPL;
    if (overlap(B, X, sizeof(double) * (size_t)P.ntot * nrhs)) { set_error("gmres_solve_block: B and X overlap"); return TSFDE_EINVAL; }
    if (!block_solver_supported(P, o)) return TSFDE_ENOTIMPL;
    tsfde_stats S{};
    tsfde_status rc = TSFDE_OK;
    TSFDE_GUARD("gmres_solve_block", rc = solve_block(P, nrhs, B, X, rel_res, o, S, (hipStream_t)stream);)
    if (stats) *stats = S;
    if (rc == TSFDE_ENOCONV) set_error("gmres_solve_block: tolerance not reached (largest rel. residual %.3e)", S.rel_res);
    return rc;
}

tsfde_status tsfde_recover_f_block(tsfde_problem* prob, int nrhs, const double* mus, double* f_out, double* rel_res,
                                   const tsfde_opts* opts, tsfde_stats* stats, void* stream) {
    if (!prob || !mus || !f_out) { set_error("recover_f_block: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    if (!check_block(P, nrhs, o, "recover_f_block")) return TSFDE_ENOTIMPL;
    if (!block_solver_supported(P, o)) return TSFDE_ENOTIMPL;
    tsfde_stats S{};
    tsfde_status rc = TSFDE_OK;
    hipStream_t st = (hipStream_t)stream;
    const long long n = P.ntot, Nd = P.Nd;
    TSFDE_GUARD("recover_f_block", {
        // right-hand sides z(mu_c) and solutions, 2 nrhs vectors held by the problem
        if (P.blk_io_cols < nrhs) {
            if (P.blk_io) {
                (void)hipFree(P.blk_io);
                P.bytes -= sizeof(double) * 2 * (size_t)n * P.blk_io_cols;
                P.blk_io = nullptr;
                P.blk_io_cols = 0;
            }
            if (o.max_device_bytes > 0 && P.bytes + sizeof(double) * 2 * (size_t)n * nrhs > (size_t)o.max_device_bytes)
                throw CapError{"max_device_bytes: no room for the right-hand sides and solutions of the block"};
            dev_alloc(P, P.blk_io, 2 * (size_t)n * nrhs);
            P.blk_io_cols = nrhs;
        }
        double* Bz = P.blk_io;
        double* Xs = P.blk_io + (size_t)n * nrhs;
        for (int c = 0; c < nrhs; ++c) launch_build_z(P, Bz + (size_t)c * n, st, mus + (size_t)c * Nd);
        launch_fill(Xs, n * nrhs, 0.0, st);
        rc = solve_block(P, nrhs, Bz, Xs, rel_res, o, S, st);
        for (int c = 0; c < nrhs; ++c)
            launch_copy<double>(Xs + (size_t)c * n + (size_t)P.M * Nd, f_out + (size_t)c * Nd, Nd, st);
        TSFDE_HIP(hipStreamSynchronize(st));
    })
    if (stats) *stats = S;
    if (rc == TSFDE_ENOCONV) set_error("recover_f_block: tolerance not reached (largest rel. residual %.3e)", S.rel_res);
    return rc;
}

// Autotuner: picks, by timing them on this problem, the 2D matvec's FFT tiling and the persistent
// P^-1 grid (kept by the problem), then the restart length and, for CG blocks, the inner tolerance
// and the warm start of recover_f (written to opts).
tsfde_status tsfde_autotune(tsfde_problem* prob, tsfde_opts* opts, int what, tsfde_tuning* out, void* stream) {
    if (!prob || !opts) { set_error("autotune: NULL argument"); return TSFDE_EINVAL; }
    if (what < 1 || what > 3) { set_error("autotune: what must be 1 (kernels), 2 (solver) or 3 (both)"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    Opts o = get_opts(opts);
    if (!check_opts(o)) return TSFDE_EINVAL;
    if (!block_solver_supported(P, o)) return TSFDE_ENOTIMPL;
    tsfde_tuning T{};
    T.mv_variant = -1;
    hipStream_t st = (hipStream_t)stream;
    auto body = [&]() {
        const long long n = P.ntot;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        TSFDE_HIP(hipEventCreate(&e0));
        TSFDE_HIP(hipEventCreate(&e1));
        struct Events {
            hipEvent_t a, b;
            ~Events() {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } ev{e0, e1};
        // milliseconds per call of fn, after one untimed call
        auto time_ms = [&](int reps, const std::function<void()>& fn) {
            fn();
            TSFDE_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) fn();
            TSFDE_HIP(hipEventRecord(e1, st));
            TSFDE_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            TSFDE_HIP(hipEventElapsedTime(&ms, e0, e1));
            return (double)ms / reps;
        };
        if (what & 1) {
            // a seeded vector and the problem's own scratch (the recover_f buffers)
            if (!P.xbuf) dev_alloc(P, P.xbuf, n);
            if (!P.rwork) dev_alloc(P, P.rwork, n);
            launch_hash_fill(P.xbuf, n, 0x5eedULL, st);
            int ids[8];
            const int nv = mv_variants(P, ids, 8);
            double best = 1e300;
            for (int i = 0; i < nv; ++i) {
                P.mv_variant = ids[i];
                const double ms = time_ms(5, [&] { apply_A_impl<double>(P, P.xbuf, P.rwork, st); });
                T.mv_ids[T.n_mv] = ids[i];
                T.mv_ms[T.n_mv++] = ms;
                if (ms < best) { best = ms; T.mv_variant = ids[i]; }
            }
            P.mv_variant = T.mv_variant;
            // the persistent P^-1 grid (2D; the block forms the persistent kernel runs)
            const bool pers = persistent_supported(P) && P.d == 2 && env_int("TSFDE_PINV", 1) != 0 &&
                              (o.block_solver == TSFDE_BLOCK_CG || (o.block_solver == TSFDE_BLOCK_TAU && tau_persistent(P)));
            if (pers) {
                int dev = 0, ncu = 0;
                TSFDE_HIP(hipGetDevice(&dev));
                TSFDE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
                const int cand[7] = {0, ncu / 16, ncu / 8 + 1, ncu / 8 * 3 / 2 + 1, ncu / 4 + 1, ncu / 8 * 3 + 1, ncu / 2};
                double bestp = 1e300;
                Opts op = o;
                launch_build_z(P, P.z_rhs, st);
                for (int c : cand) {
                    if (c < 0 || T.n_pinv >= 8) continue;
                    P.pinv_blocks = c;
                    const double ms = time_ms(2, [&] { pinv_impl<double>(P, P.z_rhs, P.rwork, op, st, true); });
                    T.pinv_cand[T.n_pinv] = c;
                    T.pinv_ms[T.n_pinv++] = ms;
                    if (ms < bestp) { bestp = ms; T.pinv_blocks = c; }
                }
                P.pinv_blocks = T.pinv_blocks;
            }
        }
        T.restart = o.restart;
        T.inner_tol = o.inner_tol;
        T.warm_start = o.warm_start;
        if (what & 2) {
            if (!P.xbuf) dev_alloc(P, P.xbuf, n);
            // seconds of a recover_f with these settings, infinite if it misses the tolerance
            auto run = [&](const Opts& oo, int* iters) {
                tsfde_stats S{};
                launch_fill(P.xbuf, n, 0.0, st);
                launch_build_z(P, P.z_rhs, st);
                TSFDE_HIP(hipStreamSynchronize(st));
                const double t0 = now();
                const tsfde_status rc = solve(P, P.z_rhs, P.xbuf, oo, S, st);
                const double dt = now() - t0;
                ++T.solves;
                if (iters) *iters = S.iters;
                return rc == TSFDE_OK ? dt : 1e300;
            };
            // the iteration count with a long cycle, then the shortest restart that holds it
            Opts c = o;
            c.restart = std::max(o.restart, 100);
            int k0 = 0;
            double best = run(c, &k0);
            int r_best = c.restart;
            if (best < 1e300 && k0 < c.restart) {
                r_best = std::min(kMaxRestart, std::max(8, k0 + 2 + k0 / 10));
            } else {
                for (int r : {50, 200}) {
                    Opts cr = o;
                    cr.restart = r;
                    const double t = run(cr, nullptr);
                    if (t < best) { best = t; r_best = r; }
                }
            }
            c.restart = r_best;
            if (o.block_solver == TSFDE_BLOCK_CG && o.use_precond) {
                double it_best = o.inner_tol;
                for (double it : {0.3, 0.1, 0.03, 0.01}) {
                    Opts ci = c;
                    ci.inner_tol = it;
                    const double t = run(ci, nullptr);
                    if (t < best) { best = t; it_best = it; }
                }
                c.inner_tol = it_best;
                int ws_best = o.warm_start;
                for (int ws : {TSFDE_WARM_PREVIOUS, TSFDE_WARM_LINEAR, TSFDE_WARM_QUADRATIC, TSFDE_WARM_HALF}) {
                    if (ws == c.warm_start) continue;
                    Opts cw = c;
                    cw.warm_start = ws;
                    const double t = run(cw, nullptr);
                    if (t < best) { best = t; ws_best = ws; }
                }
                c.warm_start = ws_best;
            }
            T.restart = c.restart;
            T.inner_tol = c.inner_tol;
            T.warm_start = c.warm_start;
            T.solve_s = best < 1e300 ? best : -1.0;
            opts->restart = c.restart;
            opts->inner_tol = c.inner_tol;
            opts->warm_start = c.warm_start;
        }
        T.pinv_blocks = P.pinv_blocks;
        T.mv_variant = P.mv_variant;
    };
    TSFDE_GUARD("autotune", body();)
    if (out) *out = T;
    return TSFDE_OK;
}

tsfde_status tsfde_recover_f_multi(tsfde_problem* const* probs, int count, double* const* f_out,
                                   const tsfde_opts* opts, tsfde_stats* stats, void* stream) {
    if (count < 0 || (count > 0 && (!probs || !f_out))) {
        set_error("recover_f_multi: count < 0 or NULL arrays");
        return TSFDE_EINVAL;
    }
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    if (o.precision != TSFDE_FP64 || o.block_solver != TSFDE_BLOCK_CG || o.recompute_z) {
        set_error("recover_f_multi: FP64, CG blocks and kept directions only");
        return TSFDE_ENOTIMPL;
    }
    std::vector<Problem*> ps;
    for (int i = 0; i < count; ++i) {
        if (!probs[i] || !f_out[i]) { set_error("recover_f_multi: NULL problem or output %d", i); return TSFDE_EINVAL; }
        for (int k = 0; k < i; ++k)
            if (probs[k] == probs[i]) { set_error("recover_f_multi: problem %d repeated", i); return TSFDE_EINVAL; }
        Problem& P = *probs[i]->p;
        if (o.use_precond && !(persistent_supported(P) && env_int("TSFDE_PINV", 1) != 0)) {
            set_error("recover_f_multi: problem %d has no persistent P^-1", i);
            return TSFDE_ENOTIMPL;
        }
        ps.push_back(&P);
    }
    if (count == 0) return TSFDE_OK;
    tsfde_status rc = TSFDE_OK;
    TSFDE_GUARD("recover_f_multi", rc = recover_multi_impl(ps, f_out, o, stats, (hipStream_t)stream);)
    if (rc == TSFDE_ENOCONV) set_error("recover_f_multi: a problem missed the tolerance (see its stats)");
    return rc;
}

tsfde_status tsfde_forward_solve(tsfde_problem* prob, const double* f, double* v, const tsfde_opts* opts,
                                 void* stream) {
    if (!prob || !f || !v) { set_error("forward_solve: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    o.block_solver = TSFDE_BLOCK_CG;  // the direct problem is solved, not preconditioned
    hipStream_t st = (hipStream_t)stream;
    TSFDE_GUARD("forward_solve", {
        if (!P.fwd_work) dev_alloc(P, P.fwd_work, 2 * (size_t)P.ntot);
        double* zh = P.fwd_work;
        double* y = P.fwd_work + P.ntot;
        launch_build_zhat(P, f, zh, st);
        pinv_impl<double>(P, zh, y, o, st, false);
        launch_copy<double>(y, v, (long long)P.M * P.Nd, st);
        TSFDE_HIP(hipStreamSynchronize(st));
    })
    return TSFDE_OK;
}

tsfde_status tsfde_apply_AT(tsfde_problem* prob, const double* lam, double* z, void* stream) {
    if (!prob || !lam || !z) { set_error("apply_AT: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    if (overlap(lam, z, sizeof(double) * P.ntot)) { set_error("apply_AT: lam and z overlap"); return TSFDE_EINVAL; }
    TSFDE_GUARD("apply_AT", apply_AT_impl(P, lam, z, (hipStream_t)stream);)
    return TSFDE_OK;
}

tsfde_status tsfde_apply_PT_inv(tsfde_problem* prob, const double* g, double* lam, const tsfde_opts* opts,
                                void* stream) {
    if (!prob || !g || !lam) { set_error("apply_PT_inv: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    if (overlap(g, lam, sizeof(double) * P.ntot)) { set_error("apply_PT_inv: g and lam overlap"); return TSFDE_EINVAL; }
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    TSFDE_GUARD("apply_PT_inv", {
        ptinv_launch(P, g, lam, o, st);
        TSFDE_HIP(hipStreamSynchronize(st));
    })
    return TSFDE_OK;
}

tsfde_status tsfde_adjoint_solve(tsfde_problem* prob, const double* g, double* lam, const tsfde_opts* opts,
                                 tsfde_stats* stats, void* stream) {
    if (!prob || !g || !lam) { set_error("adjoint_solve: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    if (overlap(g, lam, sizeof(double) * P.ntot)) { set_error("adjoint_solve: g and lam overlap"); return TSFDE_EINVAL; }
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    tsfde_stats S{};
    tsfde_status rc = TSFDE_OK;
    TSFDE_GUARD("adjoint_solve", rc = adjoint_impl(P, g, lam, o, S, (hipStream_t)stream);)
    if (stats) *stats = S;
    if (rc == TSFDE_ENOCONV) set_error("adjoint_solve: tolerance not reached (rel. residual %.3e)", S.rel_res);
    return rc;
}

tsfde_status tsfde_recover_f_vjp(tsfde_problem* prob, const double* y, const double* gf, double* grad_mu,
                                 double* grad_alpha, double* grad_gamma2, const tsfde_opts* opts, tsfde_stats* stats,
                                 void* stream) {
    if (!prob || !y || !gf) { set_error("recover_f_vjp: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    tsfde_stats S{};
    const tsfde_status rc = vjp_impl(P, y, gf, grad_mu, grad_alpha, grad_gamma2, o, S, (hipStream_t)stream);
    if (stats) *stats = S;
    return rc;
}

tsfde_status tsfde_arnoldi(tsfde_problem* prob, const double* b, int k, double* H, int* steps,
                           const tsfde_opts* opts, void* stream) {
    if (!prob || !H) { set_error("arnoldi: NULL argument"); return TSFDE_EINVAL; }
    if (k < 1 || k > kMaxRestart) { set_error("arnoldi: need 1 <= k <= %d", kMaxRestart); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    if (!block_solver_supported(P, o)) return TSFDE_ENOTIMPL;
    hipStream_t st = (hipStream_t)stream;
    const long long n = P.ntot;
    int done = 0;
    TSFDE_GUARD("arnoldi", {
        SolveOps ops;
        ops.A = [&](const double* v, double* out) { apply_A_impl<double>(P, v, out, st); };
        ops.M = [&](const double* v, double* out) -> long long {
            if (!o.use_precond) {
                launch_copy<double>(v, out, n, st);
                return 0;
            }
            return pinv_impl<double>(P, v, out, o, st, true);
        };
        if (!b) {
            launch_build_z(P, P.z_rhs, st);
            b = P.z_rhs;
        }
        done = arnoldi_impl(P, ops, b, k, H, st);
    })
    if (steps) *steps = done;
    return TSFDE_OK;
}

tsfde_status tsfde_singular_value_estimates(tsfde_problem* prob, int precond, int iters, double* sigma_max,
                                           double* sigma_min, int* iterations, const tsfde_opts* opts, void* stream) {
    if (!prob || !sigma_max || !sigma_min) { set_error("singular_value_estimates: NULL argument"); return TSFDE_EINVAL; }
    if (precond != 0 && precond != 1) { set_error("singular_value_estimates: precond must be 0 or 1"); return TSFDE_EINVAL; }
    if (iters < 1 || iters > 1000) { set_error("singular_value_estimates: iters must be in [1, 1000]"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    o.block_solver = TSFDE_BLOCK_CG;  // the preconditioner of §5.1 itself
    if (!opts) o.inner_tol = 1e-13;
    int used[2] = {0, 0};
    tsfde_status rc = TSFDE_OK;
    TSFDE_GUARD("singular_value_estimates",
                rc = singular_values_impl(P, precond, iters, *sigma_max, *sigma_min, used, o, (hipStream_t)stream);)
    if (iterations) {
        iterations[0] = used[0];
        iterations[1] = used[1];
    }
    if (rc == TSFDE_ENOCONV) set_error("singular_value_estimates: an inner solve missed its tolerance");
    return rc;
}

tsfde_status tsfde_discrepancy(tsfde_problem* prob, const double* f, double* residual, const tsfde_opts* opts,
                               void* stream) {
    if (!prob || !f || !residual) { set_error("discrepancy: NULL argument"); return TSFDE_EINVAL; }
    Problem& P = *prob->p;
    const Opts o = get_opts(opts);
    if (opts && !check_opts(o)) return TSFDE_EINVAL;
    TSFDE_GUARD("discrepancy", *residual = discrepancy_impl(P, f, o, (hipStream_t)stream);)
    return TSFDE_OK;
}

tsfde_status tsfde_ritz_values(const double* H, int ldh, int m, double* re, double* im) {
    if (!H || !re || !im || m < 1 || ldh < m) { set_error("ritz_values: need H, re, im and 1 <= m <= ldh"); return TSFDE_EINVAL; }
    try {
        std::vector<double> A((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) A[(size_t)i * m + j] = H[(size_t)i * ldh + j];
        std::vector<double> wr, wi;
        if (!hessenberg_eigenvalues(A, m, wr, wi)) {
            set_error("ritz_values: the QR iteration did not converge");
            return TSFDE_ENOCONV;
        }
        std::copy(wr.begin(), wr.end(), re);
        std::copy(wi.begin(), wi.end(), im);
    } catch (const std::bad_alloc&) {
        set_error("ritz_values: host allocation failed");
        return TSFDE_ENOMEM;
    }
    return TSFDE_OK;
}

const char* tsfde_last_error(void) { return last_error(); }

}  // extern "C"
