// Internal declarations of the tsfde library: the problem object, device buffers
// and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "tsfde.h"
#include "common.hpp"

namespace tsfde {

void set_error(const char* fmt, ...);

struct HipError {
    hipError_t code;
    std::string where;
};

#define TSFDE_HIP(call)                                                  \
    do {                                                                 \
        hipError_t e_ = (call);                                          \
        if (e_ != hipSuccess) throw ::tsfde::HipError{e_, #call};        \
    } while (0)

// Device arrays of one precision.
template <typename T>
struct Dev {
    T* gamma1 = nullptr;   // [M][Nd]
    T* gamma2 = nullptr;   // [M][Nd]
    T* dg = nullptr;       // [M][Nd]  e_0 gamma1 / gamma2 (symmetrised diagonal of block s)
    T* epad = nullptr;     // [kEpad + M] zeros then e_0..e_{M-1}
    T* q = nullptr;        // [M]
    T* sym = nullptr;      // Toeplitz circulant symbol / L^d; d=1: [L]; d=2: [H][L]
    cplx<T>* tw = nullptr;   // [L]  twiddles exp(-2 pi i m / L)
    cplx<T>* twd = nullptr;  // [Ld] twiddles for the sine transform (tau preconditioner)
    T* tau = nullptr;        // [Nd] tau eigenvalues of B (natural tau matrix); 2D: tau[k2 N + k1], k2 the
                             // frequency along the fast (last) index, so a row holds all k1 for one k2
    // work
    cplx<T>* spec = nullptr;  // [nspec_slices][H][N] (d=2) half spectra of row transforms
    T* pcg = nullptr;         // 8 vectors of Nd: x r z p q t1 t2 rhs
    T* partial = nullptr;     // block partial sums
    T* vecA = nullptr;        // scratch vectors of n_tot (mixed-mode staging)
    T* vecB = nullptr;
};

constexpr int kMaxRestart = 1000;  // largest FGMRES restart length accepted
constexpr int kHB = 16;            // time steps per history block of the forward substitution
constexpr int kArnBlocks = 4096;   // blocks of the Arnoldi sweeps
constexpr int kEpad = 256;   // leading zeros in epad (covers the history tile overhang)
constexpr int kMaxPartials = 4096;

struct Problem {
    int d = 1, N = 1, M = 1;
    double T = 1, beta = 0.5, omega = 1.5, alpha = 1e-3, length = 1;
    long long Nd = 1, ntot = 1;
    double h = 0, dt = 0, eta = 0, ct = 0, cf = 0;
    int L = 8, H = 5;     // circulant embedding length per direction (pow2 >= 2N-1), L/2+1
    int Ld = 0;           // sine-transform extension 2(N+1) when it is a power of two, else 0
    int nspec = 0;        // slices the spectrum buffer holds
    std::vector<double> stencil;  // a_l, 0 <= l_i < N, last index fastest
    std::vector<double> e, b, sigma;  // e_m, b_m, mean of dg per step
    std::vector<double> gamma1_h, gamma2_h, q_h, rho_h, mu_h;
    Dev<double> f64;
    Dev<float> f32;
    bool have_f32 = false;
    double* d_bw = nullptr;    // [M] b_0..b_{M-1}
    double* d_sigma = nullptr; // [M] sigma_s, the slice mean of e_0 gamma1 / gamma2 (tau preconditioner shift)
    double* d_rho = nullptr;   // [Nd]
    double* d_mu = nullptr;    // [Nd]
    bool tau_ok = false;       // sine-transform preconditioner available (2(N+1) a power of two)
    // 2(N+1) not a power of two: the inner CG of the persistent P^-1 is preconditioned by
    // R tau_Nt^{-1} R^T, the tau matrix of the next size Nt = 2^k - 1 > N per direction on the
    // zero-padded residual (R keeps the first N entries per direction), which is SPD; the circulant
    // embedding is then L = 2 (Nt + 1)
    bool tau_pad = false;
    int Nt = 0;                // sine-transform size of the preconditioner (N unless tau_pad)
    double a0 = 0;             // stencil centre a_0 (Jacobi fallback)
    double* z_rhs = nullptr;   // built right-hand side z (FP64, n_tot)
    double* xbuf = nullptr;    // solution buffer for recover_f (n_tot)
    // FGMRES basis storage (allocated on demand)
    double* V = nullptr;
    double* Z = nullptr;
    int basis_m = 0;
    int basis_zm = 0;            // preconditioned directions Z held (basis_m, or 1 when recomputed)
    std::vector<double> res_hist;  // relative residuals of the last solve (tsfde_stats.history)
    double* arn_part = nullptr;  // Arnoldi block partials [kArnMaxK][kArnBlocks]
    double* arn_h = nullptr;     // Arnoldi coefficients, 2 (kMaxRestart + 2) + 1
    double* rwork = nullptr;     // FGMRES residual (n_tot)
    double* adj_u = nullptr;     // adjoint work: gamma2-scaled slices (n_tot)
    double* refine_work = nullptr;  // MIXED refinement: residual, correction, inner FGMRES residual (3 n_tot)
    double* vjp_work = nullptr;     // vector-Jacobian product: [0; gf], lam, a scratch vector (3 n_tot)
    // Strang blocks (S_{n,S}), built on first use: [N] cas table then [Nd] eigenvalues of s(B)
    double* strang64 = nullptr;
    float* strang32 = nullptr;
    double strang_min = 0;       // smallest eigenvalue of s(B)
    double* strang_hist = nullptr;  // kHB slices: far history of one block of steps (FP64, or FP32 in place)
    // T_{n,S} blocks by dense sine transforms (any N), built on first use: [2(N+1)] sin table then [Nd]
    // tau eigenvalues of B
    double* taud64 = nullptr;
    float* taud32 = nullptr;
    double taud_min = 0;         // smallest tau eigenvalue
    unsigned* dense_bar = nullptr;  // barrier counter and abort word of the persistent dense block solver
    void* pw64 = nullptr;           // persistent P^{-1} work buffers (FP64 / FP32)
    void* pw32 = nullptr;
    double* fwd_work = nullptr;     // direct problem: z-hat and the substitution's output (2 n_tot)
    double* spec_work = nullptr;    // singular-value estimates: two scratch vectors and the Lanczos basis
    size_t spec_vecs = 0;           // vectors of n_tot in spec_work
    // the matvec's history sum runs on a stream of its own beside the Toeplitz passes (d = 2)
    hipStream_t mv_aux = nullptr;
    hipEvent_t mv_fork = nullptr, mv_join = nullptr;
    double* dev_scalars = nullptr;  // small device scratch (dots, flags)
    double* host_scalars = nullptr; // pinned mirror
    size_t bytes = 0;               // device bytes the problem holds (tsfde_device_bytes)
    size_t basis_bytes = 0;         // of which the FGMRES basis V, Z
    // block FGMRES (block_krylov.hip): basis and directions (vectors of a leading dimension rounded up
    // to 64), Gram partial sums, a small transfer buffer; right-hand sides and solutions of
    // tsfde_recover_f_block
    double* blk_V = nullptr;
    double* blk_part = nullptr;
    double* blk_small = nullptr;
    double* blk_io = nullptr;
    size_t blk_bytes = 0;
    int blk_nvec = 0, blk_p = 0, blk_io_cols = 0;
    // tuned settings (tsfde_autotune; built-in choices when 0 / -1): the persistent P^-1 grid (2D)
    // and the 2D matvec's FFT tiling (mv_variant_* in toeplitz2d.hip)
    int pinv_blocks = 0;
    int mv_variant = -1;
    // FGMRES restart cycles as HIP graphs (opts.graph): while capturing, the persistent P^-1 records
    // the CU slots its grid needs (graph_slots) instead of holding them, and leaves its counters to
    // the solver; the instantiated cycle, what it was captured for, its capture stream, the
    // per-step coefficients (device) and their pinned mirror
    // the transposed sweep on the persistent kernels (pinv_adjoint_run): history weights per earlier
    // step and reversed shifts while it runs; reversed right-hand sides and block weights, shifts
    bool adjoint_sweep = false;
    const double* sweep_sigma = nullptr;
    double* adj_rev = nullptr;
    // launch tables of shared P^-1 launches over several problems (device, pinned mirror)
    void* multi_dev = nullptr;
    void* multi_host = nullptr;
    size_t multi_bytes = 0;
    bool capturing = false;
    int graph_slots = 0;
    hipGraphExec_t cyc_exec = nullptr;
    hipStream_t cyc_stream = nullptr;
    unsigned long long cyc_key[10] = {};
    double* cyc_h = nullptr;
    double* cyc_h_host = nullptr;
    int cyc_len = 0;
};

// Solver options (tsfde_opts, validated)
struct Opts {
    int restart = 50, maxit = 0, precision = TSFDE_FP64, use_precond = 1, inner_maxit = 200, max_refine = 30;
    int block_solver = TSFDE_BLOCK_CG, warm_start = TSFDE_WARM_LINEAR;
    double tol = 1e-10, inner_tol = 1e-12, refine_tol = 1e-5;
    long long max_device_bytes = 0;
    int recompute_z = 0;
    int graph = 0;
};

// The two operators of a right-preconditioned Krylov solve (FP64 vectors of n_tot)
struct SolveOps {
    std::function<void(const double*, double*)> A;      // out = A v
    std::function<long long(const double*, double*)> M; // out = M v (returns inner iterations)
};

// A device-memory cap (opts.max_device_bytes) that a solve's buffers would exceed
struct CapError {
    std::string msg;
};

// Block FGMRES (block_krylov.hip): p <= kBlockMaxCols columns, basis of at most kBlockMaxBasis vectors
// per restart cycle (restart * p).  B, X: p vectors of n_tot each, contiguous; X holds the initial
// guesses.  rel receives each column's relative residual (true residual at the end of the last cycle).
constexpr int kBlockMaxCols = 16;
constexpr int kBlockMaxBasis = 1024;
size_t block_basis_bytes(const Problem& P, int p, int m);
int block_fgmres(Problem& P, const SolveOps& ops, int p, const double* B, double* X, double rtol, int restart,
                 int maxit, hipStream_t st, tsfde_stats& S, std::vector<double>& rel, bool& conv, const Opts& o);
double now_seconds();

// hipMalloc of `count` values counted against the problem's device bytes
template <typename T>
inline void dev_alloc(Problem& P, T*& ptr, size_t count) {
    void* p = nullptr;
    TSFDE_HIP(hipMalloc(&p, sizeof(T) * count));
    ptr = static_cast<T*>(p);
    P.bytes += sizeof(T) * count;
}

// ---- launchers (kernels.hip / spectral.hip) ----
template <typename T>
void launch_history_matvec(const Problem& P, const Dev<T>& D, const T* y, T* z, hipStream_t s);

// Toeplitz part of the matvec: z_s += c_t gamma2_s .* (B y_s) (s < M) and
// z_M = c_f gamma2_{M-1} .* (B y_M) + ylast (ylast null: y_{M-1}; D.gamma2 null: ones).
// d = 2 with workgroup-coalesced transposes (false if the shape is not covered), or the general path
// before_inv: an event the stream waits for before the epilogue adds to z (the history sum running on
// another stream), or null
bool toeplitz2d_supported(const Problem& P);
template <typename T>
bool launch_toeplitz2d_matvec(const Problem& P, const Dev<T>& D, const T* y, T* z, hipStream_t s,
                              const T* ylast = nullptr, hipEvent_t before_inv = nullptr);
// 2D matvec FFT tilings: 0 = 8 values per thread, length fixed at 512; 1 = 8, 2 = 16, 3 = 32 values per
// thread, run-time length; 4 = 16 values per thread, length 512.  Lists the ones that apply to P
// (at least 8 threads per transform, the workgroup's LDS within 160 KiB); returns their number.
int mv_variants(const Problem& P, int* ids, int max_ids);
template <typename T>
void launch_toeplitz_matvec(const Problem& P, const Dev<T>& D, const T* y, T* z, hipStream_t s,
                            const T* ylast = nullptr);

// q = dg .* p + c * B p  (single slice, dg may be null), with per-block partials of (p, q)
template <typename T>
void launch_spd_apply(const Problem& P, const Dev<T>& D, const T* p, T* q, const T* dg, T c,
                      T* partials, int* nparts, hipStream_t s);

// z = (2/(N+1))^d S diag(1/(sigma + c*tau)) S r with S the sine transform (tau preconditioner),
// per-block partials of (r, z)
template <typename T>
void launch_tau_prec(const Problem& P, const Dev<T>& D, const T* r, T* z, T sigma, T c,
                     T* partials, int* nparts, hipStream_t s);

// r = (z_s - gamma1_s .* sum_{m<s} e_{s-m} y_m) ./ gamma2_s  for block step s (0-based)
template <typename T>
void launch_step_rhs(const Problem& P, const Dev<T>& D, const T* z, const T* y, int s, T* rhs,
                     T scale_last, hipStream_t st);

// transposed operators (kernels.hip): the history, diagonal and f-row terms of A^T lam; the
// gamma2 scaling of all slices (only < 0), or of one slice `in` into slice `only` of out (inverse:
// division); the backward-substitution right-hand side
template <typename T>
void launch_history_adj(const Problem& P, const Dev<T>& D, const T* lam, T* z, hipStream_t s);
template <typename T>
void launch_scale_g2(const Problem& P, const Dev<T>& D, const T* in, T* out, int only, bool inverse, hipStream_t s);
template <typename T>
void launch_adj_step_rhs(const Problem& P, const Dev<T>& D, const T* g, const T* lam, int m, T* rhs, hipStream_t s);
// G (M N^d) = dL/dgamma2 from lam and v = (c_t B y^(s), s < M; c_f B y^(M))
void launch_gamma2_grad(const Problem& P, const double* lam, const double* v, double* G, hipStream_t s);

// BLAS-1 helpers
template <typename T>
void launch_dot_partials(const T* a, const T* b, long long n, T* partials, int* nparts, hipStream_t s);
template <typename T>
void launch_copy(const T* a, T* b, long long n, hipStream_t s);
void launch_d2f(const double* a, float* b, long long n, hipStream_t s);
void launch_f2d(const float* a, double* b, long long n, hipStream_t s);
void launch_sum_partials(const double* partials, int n, double* out, hipStream_t s);
void launch_sum_partials(const float* partials, int n, double* out, hipStream_t s);

// CG vector updates with device scalars: see kernels.hip
template <typename T>
void launch_cg_update_xr(T* x, T* r, const T* p, const T* q, const double* scal, long long n,
                         T* partials, int* nparts, hipStream_t s);
template <typename T>
void launch_cg_update_p(T* p, const T* z, const double* scal, long long n, hipStream_t s);
void launch_cg_scalars(double* scal, int mode, hipStream_t s);

// Arnoldi helpers (FP64), 1 <= k <= kArnMaxK basis vectors; partials holds k * nblk doubles
constexpr int kArnMaxK = 64;
void launch_multidot(const double* V, long long n, int k, const double* w, double* partials,
                     int nblk, hipStream_t s);
void launch_cgs_sub_dot(const double* V, long long n, int k, const double* h, double* w, double* partials,
                        int nblk, hipStream_t s);
void launch_cgs_sub_norm(const double* V, long long n, int k, const double* h, double* w, double* partials,
                         int nblk, hipStream_t s);
void launch_multidot_finish(const double* partials, int nblk, int k, double* h, hipStream_t s);
void launch_gemv_add(const double* Z, long long n, int k, const double* y, double* x, hipStream_t s);
void launch_scale(double* v, long long n, const double* num, const double* den, hipStream_t s);
void launch_axpby(double a, const double* x, double b, const double* y, double* out, long long n,
                  hipStream_t s);
void launch_build_z(const Problem& P, double* z, hipStream_t s, const double* mu = nullptr);  // mu: P's when null
void launch_build_zhat(const Problem& P, const double* f, double* zhat, hipStream_t s);
void launch_fill(double* p, long long n, double v, hipStream_t s);
// P v = A v + eta (q (x) I) v^(M) in the rows s < M (transpose: P^T u = A^T u + eta sum_s q_s u^(s) in
// the last block), added to out
void launch_coupling(const Problem& P, const double* v, double* out, bool transpose, hipStream_t s);
// uniform values in [-1, 1) from a hash of (seed, index)
void launch_hash_fill(double* x, long long n, unsigned long long seed, hipStream_t s);
void launch_fill(float* p, long long n, float v, hipStream_t s);
void launch_fill(unsigned long long* p, long long n, unsigned long long v, hipStream_t s);
template <typename T>
void launch_sub_partials(const T* a, const T* b, T* out, long long n, T* partials, int* nparts, hipStream_t s);
template <typename T>
void launch_jacobi_prec(const T* r, T* z, const T* dg, T c, T a0, long long n, T* partials, int* nparts,
                        hipStream_t s);

// persistent P^{-1} (pinv_persistent.hip)
bool persistent_supported(const Problem& P);
template <typename T>
long long pinv_persistent_run(Problem& P, const Dev<T>& D, void*& wptr, const T* z, T* y, double inner_tol,
                              int inner_maxit, bool last_block, int extrap, int tblocks, hipStream_t st);
template <typename T>
void pinv_persistent_free(void* wptr);
// The same FP64 forward substitution with every work buffer in the library's static device scratch
// (tsfde_apply_P_inv_noalloc): allocates nothing.  pinv_noalloc_bytes is the scratch the problem
// needs, kNoAllocScratchBytes what the scratch holds.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
size_t pinv_noalloc_bytes(const Problem& P);
long long pinv_persistent_run_noalloc(Problem& P, const double* z, double* y, double inner_tol, int inner_maxit,
                                      int extrap, int tblocks, hipStream_t st);
void set_persistent_blocks(int g);
// counters of the persistent P^-1 when it runs inside a captured graph: zero the iteration count and
// the abort word before a replay; after it, read both (synchronises st; throws if a barrier wait
// timed out) and return the iterations
void pinv_graph_prepare(Problem& P, bool f32, hipStream_t st);
// y_i = P_i^{-1} z_i for several problems in shared persistent launches (FP64, CG blocks, every problem
// with persistent_supported): problems of one kernel form share a launch (2D: the same values per
// thread; 1D: also the same transform length); iters_i receives each problem's CG iterations
struct PinvMultiJob {
    Problem* P;
    const double* z;
    double* y;
    long long iters;
};
void pinv_multi_run(std::vector<PinvMultiJob>& jobs, double inner_tol, int inner_maxit, int extrap, hipStream_t st);
long long pinv_adjoint_run(Problem& P, const double* zrev, const double* dgrev, const double* sigrev, double* urev,
                           double inner_tol, int inner_maxit, int extrap, hipStream_t st);
// P^{-T} sweep helpers (kernels.hip): zrev_k = g_{M-1-k} (k = 0 also minus lam_M), dgrev_k =
// dg_{M-1-k}; then lam_m = urev_{M-1-m} / gamma2_m for m < M, in place (urev in lam's first M slices)
void launch_adj_reverse(const Problem& P, const double* g, const double* lam, double* zrev, double* dgrev,
                        hipStream_t s);
void launch_adj_unreverse(const Problem& P, double* lam, hipStream_t s);
long long pinv_graph_finish(Problem& P, bool f32, hipStream_t st);
// v *= 1 / sqrt(*sq), or v = 0 when *sq is not a positive finite number
void launch_scale_rsqrt(double* v, long long n, const double* sq, hipStream_t s);
// Batch mode of the calling thread: its persistent kernels are ordinary launches sized so that
// kMaxInflight of them fit the device together (tsfde_recover_f_batch)
constexpr int kMaxInflight = 8;
// XCDs of the device (MI355X: 8 XCDs of 32 CUs); the workgroups of a dispatch are dealt to them in turn
constexpr int kXcds = 8;
void set_shared_launch(bool on);
bool shared_launch();
void set_persistent_fixed_length(bool on);

// S_{n,S} (strang.hip): the cas table and eigenvalues of Strang's circulant (setup.hip; returns the
// smallest eigenvalue); whether the Hartley passes fit the LDS; the tables on the device (first
// use); y = S^{-1} z by forward substitution with one exact circulant solve per block
double strang_tables(const Problem& P, std::vector<double>& cas, std::vector<double>& lam);
bool strang_supported(const Problem& P);
void ensure_strang(Problem& P);
// T_{n,S} by the same dense passes with the sine transform (any N, d = 1, 2): tables (setup.hip),
// whether the passes fit the LDS, the tables on the device (first use), y = T^{-1} z
double tau_dense_tables(const Problem& P, std::vector<double>& tab, std::vector<double>& lam);
bool tau_dense_supported(const Problem& P);
void ensure_tau_dense(Problem& P);
template <typename T>
void pinv_tau_dense(Problem& P, const Dev<T>& D, const T* z, T* y, bool last_block, hipStream_t st);
template <typename T>
void pinv_strang(Problem& P, const Dev<T>& D, const T* z, T* y, bool last_block, hipStream_t st);
// w[i] = (z_s - gamma1_s sum_{m < sa} e_{s-m} y_m) / gamma2_s for s = sa + i, i < cnt <= kHB
// (pinv_persistent.hip; the far part of the history, shared with the persistent P^-1)
template <typename T>
void launch_far_history(const Problem& P, const Dev<T>& D, const T* y, T* w, const T* z, int sa, int cnt,
                        hipStream_t st);  // use the fixed-length 2D sine-transform kernels where available

}  // namespace tsfde
