/*
 * tsfde.h -- C ABI of the MI355X (gfx950) solver for the quasi-boundary-value
 * inverse source problem of a time-space fractional diffusion equation
 * (Majumdar, Serra-Capizzano, Sormani, arXiv 2507.02809).
 *
 * The library solves the all-at-once system  A y = z  of §5 (eq. lin-syst)
 * with flexible GMRES, right-preconditioned by the block lower-triangular
 * matrix P of §5.1, and returns the regularised source f~ (the last block of y).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Grid (§4): Omega = (0, length)^d, n = N interior points per direction,
 *    h = length/(N+1), x_j = j h; t_s = s T/M, s = 1..M (M is the paper's S).
 *  - Vector layout (§5, eq. lin-syst; multi-index rule of §2): a solution or
 *    right-hand side has (M+1) * N^d entries: M slices v^(1..M) followed by
 *    f~, slice-major; inside a slice the multi-index (j_1, .., j_d) runs with
 *    the LAST index fastest.
 *  - Ownership: create functions COPY their host arrays into device memory
 *    owned by the problem; the caller may free its arrays on return.  Every
 *    other pointer argument is a caller-owned DEVICE pointer unless stated
 *    otherwise; the library never retains it after the call returns.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued on it; entry points that report statistics synchronise it.
 *  - Errors: every function returns a tsfde_status; nothing is thrown across
 *    the ABI.  tsfde_last_error() returns a thread-local message describing
 *    the last failure.  On error, output buffers hold unspecified values.
 *  - Calls that share one problem object must not overlap (the problem owns
 *    its work buffers); different problem objects are independent.
 */
#ifndef TSFDE_H
#define TSFDE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsfde_problem tsfde_problem; /* opaque, library-owned */

typedef enum {
    TSFDE_OK = 0,
    TSFDE_EINVAL = 1,     /* invalid argument (parameter range, NULL, aliasing)   */
    TSFDE_ENOMEM = 2,     /* device allocation failed or exceeded max_device_bytes */
    TSFDE_EDEVICE = 3,    /* a HIP runtime call failed                             */
    TSFDE_ENOCONV = 4,    /* solver hit maxit; x holds the last iterate            */
    TSFDE_ENONFINITE = 5, /* NaN or Inf in an input array                          */
    TSFDE_ENOTIMPL = 6    /* combination not supported by this build               */
} tsfde_status;

typedef enum { TSFDE_FP64 = 0, TSFDE_MIXED = 1, TSFDE_PREC_F32 = 2 } tsfde_precision;

/* Solver options.  tsfde_default_opts() fills the defaults listed here. */
typedef struct tsfde_opts {
    int restart;         /* FGMRES restart length m                       (50)   */
    int maxit;           /* max outer iterations (all restarts, all refinement
                            sweeps together); <= 0 means min(n_tot, 1000)  (0)   */
    double tol;          /* stop when ||b - A x||_2 <= tol ||b||_2        (1e-10) */
    int precision;       /* TSFDE_FP64: every operator application in FP64;
                            TSFDE_MIXED: A and P^{-1} inside FGMRES in FP32, the
                            residual b - A x, Arnoldi, Givens and the update in
                            FP64, closed by iterative refinement;
                            TSFDE_PREC_F32: FGMRES, A, Arnoldi and Givens in FP64
                            and only P^{-1} applied in FP32 (a flexible, inexact
                            preconditioner; inner_tol is raised to >= 1e-6)
                                                                        (FP64)  */
    int use_precond;     /* 1: right preconditioning by P of §5.1; 0: none (1)   */
    double inner_tol;    /* relative residual of each diagonal-block solve inside
                            P^{-1} (preconditioned CG)                  (1e-12) */
    int inner_maxit;     /* cap on CG iterations per block solve        (200)   */
    double refine_tol;   /* MIXED: relative tolerance of each inner FGMRES
                            sweep on A d = r                            (1e-5)  */
    int max_refine;      /* MIXED: max refinement sweeps                (30)    */
    int block_solver;    /* TSFDE_BLOCK_CG: each diagonal block of P solved by
                            tau-preconditioned CG to inner_tol (P of §5.1);
                            TSFDE_BLOCK_TAU: the T_{n,S} variant of the §5.1
                            Remark -- B replaced by its tau matrix and the block's
                            coefficient ratio gamma1/gamma2 frozen at its slice
                            mean, so each block is solved exactly by sine
                            transforms (no inner iterations, no warm start), for
                            d = 1, 2 and any N: FFT-based inside the persistent
                            kernels when d = 2 and 2(N+1) is a power of two,
                            dense sine-transform passes otherwise (ENOTIMPL if
                            those do not fit the LDS, N above ~6700 in 1D and
                            ~3300 in 2D, or the tau matrix is not positive
                            definite).
                            TSFDE_BLOCK_STRANG: the S_{n,S} variant of the same
                            Remark -- B replaced by Strang's circulant (the
                            central diagonals of B wrapped around, per level),
                            the ratio frozen as above, each block solved exactly
                            by real Hartley transforms of any size N (d = 1, 2;
                            ENOTIMPL if that circulant is not positive definite,
                            which a user-supplied stencil can cause)
                                                                        (CG)    */
    int warm_start;      /* initial guess of each block CG in P^{-1} from the
                            solution of the previous time levels:
                            TSFDE_WARM_PREVIOUS (y^(s-1)), TSFDE_WARM_LINEAR
                            (2 y^(s-1) - y^(s-2)), TSFDE_WARM_QUADRATIC,
                            TSFDE_WARM_HALF (1.5 y^(s-1) - 0.5 y^(s-2)).  The
                            persistent P^{-1} applies it; the multi-launch path
                            always starts from y^(s-1)              (LINEAR) */
    long long max_device_bytes; /* cap on the device memory of the problem's arrays
                            plus the FGMRES basis (0: none).  If keeping the m
                            preconditioned directions z_j would exceed it, they
                            are recomputed (z_j = P^{-1} v_j again at the end of
                            each cycle; P^{-1} is deterministic, so the same
                            directions return); if even the basis V does not fit,
                            the solve returns TSFDE_ENOMEM            (0)     */
    int recompute_z;     /* 1: recompute the z_j at the end of each cycle instead
                            of keeping them (halves the basis memory, adds m
                            P^{-1} applications per cycle)              (0)     */
    int graph;           /* 1: run each FGMRES restart cycle (FP64 or PREC_F32,
                            persistent P^{-1} or none) as one HIP graph: the m
                            Arnoldi steps with no host round trip, captured on
                            first use, kept by the problem and replayed for later
                            cycles and solves with the same settings; the host
                            then applies the Givens rotations and takes the
                            first k <= m steps that meet tol.  Steps after
                            convergence in the last cycle are wasted work, so
                            restart should be near the iteration count
                            (tsfde_autotune).  Other settings: ignored  (0) */
} tsfde_opts;

typedef enum { TSFDE_BLOCK_CG = 0, TSFDE_BLOCK_TAU = 1, TSFDE_BLOCK_STRANG = 2 } tsfde_block_solver;
typedef enum {
    TSFDE_WARM_PREVIOUS = 0,
    TSFDE_WARM_LINEAR = 1,
    TSFDE_WARM_QUADRATIC = 2,
    TSFDE_WARM_HALF = 3
} tsfde_warm_start;

/* Statistics of a solve.  Times are wall-clock seconds on the host, measured
   around stream-synchronised phases. */
typedef struct tsfde_stats {
    int iters;                 /* outer (Arnoldi) iterations, all sweeps        */
    int restarts;              /* FGMRES restarts                               */
    int refinements;           /* MIXED: refinement sweeps (FP64: 1)            */
    int converged;             /* 1 if ||b - A x|| <= tol ||b|| was reached     */
    long long inner_iters;     /* CG iterations inside all P^{-1} applications  */
    double rel_res;            /* final ||b - A x||_2 / ||b||_2, FP64 A         */
    double t_total;            /* seconds in the solve                          */
    double t_precond;          /* seconds applying P^{-1}                       */
    double t_matvec;           /* seconds applying A                            */
    double t_ortho;            /* seconds in Gram-Schmidt and the x update      */
    int history_len;           /* entries of history                            */
    const double* history;     /* relative residuals as the solve saw them: the
                                  true one at every (re)start, the least-squares
                                  estimate after every Arnoldi step (MIXED: each
                                  sweep relative to its own right-hand side).
                                  Host memory owned by the problem, valid until
                                  its next solve or its destruction            */
} tsfde_stats;

void tsfde_default_opts(tsfde_opts* opts);

/*
 * Create a problem on the current HIP device (§4 eq. numer-scheme, §5 eq. lin-syst).
 *   d         spatial dimension, 1 or 2
 *   N         interior grid points per direction (N >= 1)
 *   M         time steps (the paper's S, M >= 1);  T > 0 final time
 *   beta      Caputo order, 0 < beta < 1 (§1)
 *   omega     fractional-Laplacian order, 1 < omega < 2 (§1)
 *   alpha     quasi-boundary regularisation parameter (the paper's lambda), > 0 (§3)
 *   gamma1    host [M][N^d], gamma_1(x_j, t_s), s = 1..M, must be >= 0
 *   gamma2    host [M][N^d], gamma_2(x_j, t_s), must be > 0
 *   q         host [M], q(t_s) > 0
 *   rho       host [N^d] initial state, or NULL for zero
 *   mu        host [N^d] noisy final-time data mu_eps, or NULL for zero
 *   out       receives the problem handle
 * Omega = (0,1)^d.  Returns EINVAL for out-of-range parameters, ENONFINITE for
 * NaN/Inf inputs, ENOMEM / EDEVICE on device failures.
 */
tsfde_status tsfde_create_problem(int d, int N, int M, double T, double beta, double omega,
                                  double alpha, const double* gamma1, const double* gamma2,
                                  const double* q, const double* rho, const double* mu,
                                  tsfde_problem** out);

/*
 * As tsfde_create_problem with Omega = (0, length)^d (the paper's experiments use
 * length = pi, §6) and an optional stencil override: `stencil` (host, N^d values,
 * a_l for 0 <= l_i <= N-1, last index fastest) replaces the library's own
 * Fourier coefficients of eq. fourier-coeff; NULL computes them (d = 1: eq.
 * fourier-coeff-1d through Lemma 1; d = 2: FFT of the sampled generating
 * function with Richardson extrapolation, the FFT route named in §4).
 */
tsfde_status tsfde_create_problem_ex(int d, int N, int M, double T, double beta, double omega,
                                     double alpha, const double* gamma1, const double* gamma2,
                                     const double* q, const double* rho, const double* mu,
                                     double length, const double* stencil, tsfde_problem** out);

/* Replace mu_eps (host [N^d]) without rebuilding the problem. */
tsfde_status tsfde_set_mu(tsfde_problem* prob, const double* mu);

/* Replace the gamma2 samples (host [M][N^d], gamma_2(x_j, t_s) > 0; §4 eq. numer-scheme)
 * without rebuilding the problem: the device copies of gamma2, of the symmetrised
 * diagonal e_0 gamma1/gamma2 of every block of P and of its slice means are refreshed.
 * Returns EINVAL for a sample <= 0, ENONFINITE for NaN/Inf. */
tsfde_status tsfde_set_gamma2(tsfde_problem* prob, const double* gamma2);

/* Replace the regularisation parameter alpha (> 0; §3): only c_f = alpha/h^omega
 * of the last block row changes, so nothing is rebuilt (a sweep over alpha
 * for a parameter choice rule reuses one problem). */
tsfde_status tsfde_set_alpha(tsfde_problem* prob, double alpha);

void tsfde_destroy_problem(tsfde_problem* prob);

/* (M+1) * N^d, the length of y and z. */
size_t tsfde_vector_length(const tsfde_problem* prob);

/* Device bytes the problem holds now: its arrays, the work buffers its calls have
   allocated so far and the FGMRES basis (opts.max_device_bytes caps this total). */
size_t tsfde_device_bytes(const tsfde_problem* prob);

/* Scalars of the discretisation: out[0] = h, out[1] = dt, out[2] = eta = dt^beta Gamma(2-beta),
   out[3] = eta/h^omega, out[4] = alpha/h^omega, out[5] = circulant embedding size L. */
tsfde_status tsfde_problem_scalars(const tsfde_problem* prob, double out[6]);

/* Copy the stencil table a_l, 0 <= l_i <= N-1 (N^d values) used by the problem into
   host memory `out` (§4 eq. fourier-coeff). */
tsfde_status tsfde_get_stencil(const tsfde_problem* prob, double* out);

/* Compute the stencil table a_l, 0 <= l_i <= N-1 (host, N^d doubles) for dimension d and
   order omega without creating a problem (host computation only). */
tsfde_status tsfde_compute_stencil(int d, int N, double omega, double* out);

/*
 * z = A y  (§5 'Implementation': time-history sum with the e_m weights scaled by D_1^(s),
 * Toeplitz product (eta/h^omega) D_2^(s) B y^(s) through a zero-padded circulant
 * embedding and FFTs, minus eta q^(s) y^(M+1); last block (alpha/h^omega) D_2^(M) B y^(M+1)
 * + y^(M)).  y, z: device, (M+1) N^d entries, must not overlap.
 */
tsfde_status tsfde_apply_A(tsfde_problem* prob, const double* y, double* z, void* stream);
tsfde_status tsfde_apply_A_f32(tsfde_problem* prob, const float* y, float* z, void* stream);

/*
 * Persistent kernels.  P^{-1} runs as persistent grids whose workgroups wait for each other at
 * device-wide barriers.  Every such grid of the process takes its share of the device's CU slots
 * before it starts and gives it back when it has finished, so that grids running side by side on
 * different streams or host threads are always resident together (a call waits on the host while
 * the slots are taken).  A barrier wait is bounded (TSFDE_BARRIER_TIMEOUT_US, default 5 s): if it
 * expires, every workgroup leaves the grid normally and the call returns TSFDE_EDEVICE.  The entry
 * points that apply P^{-1} synchronise their stream.
 *
 * y ~= P^{-1} z by the forward substitution of §5.1: for s = 1..M solve
 * (e_0 D_1^(s) + (eta/h^omega) D_2^(s) B) y^(s) = z^(s) - D_1^(s) sum_{m<s} e_{s-m} y^(m),
 * then (alpha/h^omega) D_2^(M) B y^(M+1) = z^(M+1) - y^(M).  Each block is solved by
 * preconditioned CG on its symmetrised form to opts->inner_tol (the paper uses a direct
 * solve; see the design notes).  opts may be NULL (defaults).  z, y: device, no overlap.
 */
tsfde_status tsfde_apply_P_inv(tsfde_problem* prob, const double* z, double* y,
                               const tsfde_opts* opts, void* stream);
tsfde_status tsfde_apply_P_inv_f32(tsfde_problem* prob, const float* z, float* y,
                                   const tsfde_opts* opts, void* stream);

/*
 * tsfde_apply_P_inv without device allocations, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operation, options and kernels as tsfde_apply_P_inv, but
 * the work buffers of the forward substitution live in a static device array of
 * 32 MiB that the library holds on every device it runs on until the process ends
 * (about 216 bytes per grid point of a slice: N^d up to about 150 000; 2D N = 255
 * needs 14.6 MB).  The call allocates nothing: no hipMalloc, hipFree or allocating
 * library routine.  The problem's own arrays come from tsfde_create_problem.
 *   z, y   device, (M+1) N^d, must not overlap; the call synchronises `stream`
 *   opts   as tsfde_apply_P_inv; TSFDE_BLOCK_STRANG returns TSFDE_ENOTIMPL (its
 *          tables are built on first use), as do shapes without the persistent
 *          kernels (circulant embedding L > 8192)
 * Returns TSFDE_ENOMEM, with the sizes in the message, when the problem needs more
 * than the static array holds.  Calls on one device share that array (it keeps the
 * last call's contents; the call clears what must start at zero): concurrent calls
 * on one device are serialised by the library, so overlapping calls from several
 * host threads wait for each other.
 */
tsfde_status tsfde_apply_P_inv_noalloc(tsfde_problem* prob, const double* z, double* y,
                                       const tsfde_opts* opts, void* stream);

/*
 * Solve A x = b by right-preconditioned flexible GMRES(m) (§5: GMRES with P of §5.1).
 *   b      device, (M+1) N^d; NULL uses the system's own right-hand side z of eq. lin-syst
 *   x      device, (M+1) N^d; in: initial guess, out: solution (last iterate on ENOCONV)
 *   opts   NULL for defaults;  stats  may be NULL.
 * Returns TSFDE_ENOCONV if tol was not reached within maxit.
 */
tsfde_status tsfde_gmres_solve(tsfde_problem* prob, const double* b, double* x,
                               const tsfde_opts* opts, tsfde_stats* stats, void* stream);

/*
 * Recover the regularised source: build z (eq. lin-syst), solve from x0 = 0 (§6) and write
 * f~ = y^(M+1) into f_out (device, N^d).  `work` is a device buffer of (M+1) N^d doubles
 * that receives the full solution y, or NULL to use an internal buffer.
 */
tsfde_status tsfde_recover_f(tsfde_problem* prob, double* f_out, double* work,
                             const tsfde_opts* opts, tsfde_stats* stats, void* stream);

/*
 * Recover f~ for several independent problems (the batched form of
 * tsfde_recover_f, e.g. many instances, regularisation parameters or data
 * sets).  Up to max_inflight problems (1..8) are solved at the same time,
 * each on a non-blocking stream the library creates for it, by as many host
 * worker threads (the calling thread is one of them).  Because one problem's
 * preconditioner is a chain of dependent time steps that occupies only a
 * part of the device, solving several side by side raises the throughput.
 * Their kernels overlap only as far as the HIP runtime gives the streams
 * hardware queues of their own (GPU_MAX_HW_QUEUES, 4 by default, shared with
 * every other stream of the process).
 *   probs   count distinct problem handles (on the current HIP device)
 *   f_out   count device pointers, f_out[i] receives N_i^d values
 *   opts    one set of options for all problems (NULL for defaults)
 *   stats   NULL, or count entries receiving each problem's statistics
 *   stream  work already queued on it is finished before the batch starts;
 *           every output is complete when the call returns
 * Returns EINVAL for a NULL entry, a repeated problem or max_inflight out of
 * range, ENOTIMPL if the options do not apply to one of the problems, the
 * first device error by problem index, else ENOCONV if any problem missed
 * the tolerance (its stats tell which; its f~ is the last iterate).
 */
tsfde_status tsfde_recover_f_batch(tsfde_problem* const* probs, int count, double* const* f_out,
                                   const tsfde_opts* opts, tsfde_stats* stats, int max_inflight,
                                   void* stream);

/*
 * Several right-hand sides of one problem (§5, eq. lin-syst: A X = B, e.g. the same instance with
 * several data sets mu): block flexible GMRES.  One block Krylov space of nrhs vectors per step
 * serves all columns; P^{-1} (§5.1) is applied to each column, the block Gram-Schmidt products
 * V^T W and V H run on the FP64 matrix cores, the block Hessenberg matrix is reduced by Givens
 * rotations on the host.  A restart cycle of opts.restart steps holds (restart + 1) nrhs basis and
 * restart nrhs preconditioned vectors, each (M+1) N^d doubles rounded up to a multiple of 64
 * (counted against opts.max_device_bytes).
 *   nrhs     1..16, with restart * nrhs <= 1024
 *   B        device, nrhs vectors of (M+1) N^d, contiguous (column c at B + c (M+1) N^d)
 *   X        device, same layout; in: initial guesses, out: solutions (last iterates on ENOCONV)
 *   rel_res  host, nrhs values receiving each column's true relative residual, or NULL
 *   opts     tol applies to every column; precision FP64 or PREC_F32 (MIXED: ENOTIMPL);
 *            maxit counts block steps
 * stats->iters counts block steps and stats->rel_res is the largest column residual.
 * Returns EINVAL for NULL or overlapping B, X; ENOTIMPL for nrhs or restart out of range.
 */
tsfde_status tsfde_gmres_solve_block(tsfde_problem* prob, int nrhs, const double* B, double* X,
                                     double* rel_res, const tsfde_opts* opts, tsfde_stats* stats,
                                     void* stream);

/*
 * tsfde_recover_f for nrhs data sets of the same problem in one block solve: z(mu_c) built for each
 * column (eq. lin-syst), X from zero, f~_c = the last block of column c.
 *   mus      device, nrhs x N^d (mu_c at mus + c N^d); the problem's own mu is not used
 *   f_out    device, nrhs x N^d
 * The right-hand sides and solutions (2 nrhs vectors of (M+1) N^d) are held by the problem.
 */
tsfde_status tsfde_recover_f_block(tsfde_problem* prob, int nrhs, const double* mus, double* f_out,
                                   double* rel_res, const tsfde_opts* opts, tsfde_stats* stats,
                                   void* stream);

/*
 * Autotuner: settings picked by timing them on this problem (on `stream`, with the problem's own
 * data mu), kept for its later calls or written back to opts.
 *   what = 1  kernels: the 2D matvec's FFT tiling (tsfde_tuning.mv_ids: 0 = 8 values per thread
 *             with the length fixed at 512, 1 / 2 / 3 = 8 / 16 / 32 values per thread at any
 *             length, 4 = 16 values per thread at 512), and the grid of the persistent P^{-1}
 *             kernel (2D; 0 = the built-in choice); both kept by the problem
 *   what = 2  solver: recover_f from x0 = 0 with opts' tol, precision and block_solver, once with a
 *             restart of at least 100 to learn the iteration count k (restart then k + 2 + k/10,
 *             else the faster of 50 and 200), then, for CG blocks, inner_tol in {0.3, 0.1, 0.03,
 *             0.01} and each warm start; the fastest converged setting goes to opts->restart,
 *             opts->inner_tol and opts->warm_start
 *   what = 3  both, kernels first
 * out (may be NULL) receives every timing.  About 2 + 9 solves for what = 3 with CG blocks.
 */
typedef struct tsfde_tuning {
    int mv_variant;            /* chosen matvec tiling (-1: not a 2D FFT matvec)     */
    int n_mv;                  /* tilings timed                                     */
    int mv_ids[8];
    double mv_ms[8];           /* milliseconds per apply_A                          */
    int pinv_blocks;           /* chosen P^{-1} grid (0: built-in)                  */
    int n_pinv;                /* grids timed                                       */
    int pinv_cand[8];
    double pinv_ms[8];         /* milliseconds per apply_P_inv                      */
    int restart;               /* chosen solver settings                            */
    double inner_tol;
    int warm_start;
    double solve_s;            /* seconds of the fastest timed solve (-1: none)     */
    int solves;                /* solves timed                                      */
} tsfde_tuning;

tsfde_status tsfde_autotune(tsfde_problem* prob, tsfde_opts* opts, int what, tsfde_tuning* out,
                            void* stream);

/*
 * tsfde_recover_f for several problems in lockstep, their P^{-1} applications sharing persistent
 * launches: at each Arnoldi step one launch per block of 16 time steps runs the forward
 * substitution of every unfinished problem side by side (each on its own share of the grid, with
 * its own device-wide barrier); problems of one kernel form share a launch (2D: the same values
 * per thread; 1D: also the same FFT length), launches take as many problems as fit the device's CU
 * slots together.  Matvecs, Gram-Schmidt and the Givens rotations stay per problem (stream and
 * host).  FP64 with CG blocks only (ENOTIMPL otherwise, and for a problem without the persistent
 * P^{-1}); EINVAL for NULL entries or a repeated problem; ENOCONV if any problem missed tol.
 */
tsfde_status tsfde_recover_f_multi(tsfde_problem* const* probs, int count, double* const* f_out,
                                   const tsfde_opts* opts, tsfde_stats* stats, void* stream);

/*
 * Direct problem of §6.1: v = A-hat^{-1} z-hat with z-hat^(s) = b_{s-1} D_1^(s) rho + eta q^(s) f,
 * i.e. the first M steps of the forward substitution (used to synthesise mu).
 *   f    device, N^d        v  device, M N^d (slices v^(1..M)); mu = v^(M)
 */
tsfde_status tsfde_forward_solve(tsfde_problem* prob, const double* f, double* v,
                                 const tsfde_opts* opts, void* stream);

/*
 * Transposed problem (gradients of f~ with respect to the data and the
 * regularisation parameter).  With w^(s) = gamma1^(s) .* lam^(s) and the
 * blocks of A (§5, eq. lin-syst) transposed (B is symmetric):
 *   (A^T lam)^(s) = e_0 w^(s) + sum_{r>s, r<=M} e_{r-s} w^(r) + [s = M] lam^(M+1)
 *                   + (eta/h^omega) B (gamma2^(s) .* lam^(s)),           s = 1..M
 *   (A^T lam)^(M+1) = -eta sum_s q^(s) lam^(s) + c_f B (gamma2^(M) .* lam^(M+1))
 * (1-based slices as in §5; the history sum runs backwards in time).
 * lam, z, g: device, (M+1) N^d, layout of every solution vector.
 */
tsfde_status tsfde_apply_AT(tsfde_problem* prob, const double* lam, double* z, void* stream);

/*
 * lam = P^{-T} g: backward substitution over the block rows of P^T (§5.1
 * transposed): the last block c_f B D_2^(M) lam^(M+1) = g^(M+1), then for
 * s = M..1 the block (e_0 D_1^(s) + (eta/h^omega) B D_2^(s)) lam^(s) = r^(s),
 * solved in u = D_2^(s) lam^(s) by the same SPD block CG as P^{-1}
 * (opts.inner_tol, opts.inner_maxit; FP64, one launch per CG phase).
 * g and lam must not overlap.
 */
tsfde_status tsfde_apply_PT_inv(tsfde_problem* prob, const double* g, double* lam,
                                const tsfde_opts* opts, void* stream);

/*
 * Solve A^T lam = g by flexible GMRES right-preconditioned by P^{-T} (FP64;
 * opts.precision and opts.block_solver do not apply).  lam holds the initial
 * guess.  Returns ENOCONV if opts.tol was not reached.
 */
tsfde_status tsfde_adjoint_solve(tsfde_problem* prob, const double* g, double* lam,
                                 const tsfde_opts* opts, tsfde_stats* stats, void* stream);

/*
 * Vector-Jacobian product of f~ = R A^{-1} z (R: the last block) for a loss
 * with gradient gf = dL/df~ (device, N^d), given the solution y of A y = z
 * (device, (M+1) N^d, e.g. the `work` buffer of tsfde_recover_f):
 *   lam = A^{-T} [0; gf]                           (tsfde_adjoint_solve)
 *   grad_mu    = lam^(M+1)                         (z^(M+1) = mu_eps)
 *   grad_alpha = -lam^T (dA/dalpha) y = -(c_f/alpha) lam^(M+1) . (gamma2^(M) .* B y^(M+1))
 *   grad_gamma2^(s) = -(eta/h^omega) lam^(s) .* B y^(s),  s = 1..M, and for s = M also
 *                     -c_f lam^(M+1) .* B y^(M+1)   (gamma2^(s) enters the diagonal blocks and,
 *                     at s = M, the last one)
 * grad_mu: device N^d or NULL; grad_alpha: HOST double or NULL; grad_gamma2:
 * device M N^d (slice-major like gamma2) or NULL.  The first call allocates
 * three work vectors of (M+1) N^d that the problem keeps.
 */
tsfde_status tsfde_recover_f_vjp(tsfde_problem* prob, const double* y, const double* gf,
                                 double* grad_mu, double* grad_alpha, double* grad_gamma2,
                                 const tsfde_opts* opts, tsfde_stats* stats, void* stream);

/*
 * tsfde_recover_f_vjp for several problems side by side, as tsfde_recover_f_batch
 * runs tsfde_recover_f (same worker streams, ordering, limits and status rules).
 *   ys           count device solutions of A y = z, or NULL (or a NULL entry) for
 *                the solution the problem's last tsfde_recover_f without a work
 *                buffer left in its internal buffer (EINVAL if there is none)
 *   gfs          count device gradients dL/df~ (N_i^d)
 *   grad_mu      NULL, or count device outputs (N_i^d; NULL entries skip)
 *   grad_alpha   NULL, or a HOST array of count doubles
 *   grad_gamma2  NULL, or count device outputs (M_i N_i^d; NULL entries skip)
 */
tsfde_status tsfde_recover_f_vjp_batch(tsfde_problem* const* probs, int count,
                                       const double* const* ys, const double* const* gfs,
                                       double* const* grad_mu, double* grad_alpha,
                                       double* const* grad_gamma2, const tsfde_opts* opts,
                                       tsfde_stats* stats, int max_inflight, void* stream);

/*
 * Spectral estimate of the preconditioned operator: k steps of Arnoldi
 * (classical Gram-Schmidt applied twice, as in the solver) on A P^{-1} from b
 * (device, (M+1) N^d; NULL for z of eq. lin-syst), with P^{-1} applied as in
 * tsfde_gmres_solve (opts.use_precond = 0: A itself).  H (host) receives the
 * (k+1) x k upper Hessenberg matrix, row-major; *steps the steps taken (fewer
 * than k after an exact breakdown).  The eigenvalues of its leading steps x
 * steps block are Ritz values of A P^{-1}, which has the spectrum of P^{-1} A
 * (§5.1: P^{-1} A - I has rank at most N^d, so its eigenvalues cluster at 1).
 * Uses the problem's Krylov basis storage; 1 <= k <= 1000.
 */
tsfde_status tsfde_arnoldi(tsfde_problem* prob, const double* b, int k, double* H, int* steps,
                           const tsfde_opts* opts, void* stream);

/*
 * Ritz values: the eigenvalues of the leading m x m block of a Hessenberg matrix H (host,
 * row-major with leading dimension ldh >= m, e.g. the (k+1) x k output of tsfde_arnoldi with
 * ldh = k), by Francis' double-shift QR iteration on the host.  re, im: host, m values each.
 * Returns ENOCONV if the iteration does not converge.  Needs no device.
 */
tsfde_status tsfde_ritz_values(const double* H, int ldh, int m, double* re, double* im);

/*
 * Estimates of the extreme singular values of M = A (precond = 0) or M = P^{-1} A (precond = 1),
 * whose ratio sigma_max / sigma_min is the 2-norm condition number that the tables of §6.1.1 and
 * §6.2 print: sigma_max^2 is the largest eigenvalue of M^T M and 1/sigma_min^2 that of
 * M^{-1} M^{-T}, each found by Lanczos with full reorthogonalisation (the largest Ritz value),
 * with M^{-1} = A^{-1} P and M^{-T} = P^T A^{-T} applied by FGMRES solves with A and A^T to
 * opts->tol.  P^{-1} and P^{-T} must act as fixed linear operators: they are applied with
 * opts->inner_tol (1e-13 when opts is NULL); opts->block_solver is ignored (P of §5.1).  Each
 * Lanczos run stops when its estimate changes by less than 1e-12 relative in two consecutive
 * steps, or after iters steps (1..1000); iterations (host, 2 ints, may be NULL) receives the steps
 * taken.  The estimates approach the extremes from inside: sigma_max from below, sigma_min from
 * above.  FP64.  The call keeps iters + 3 work vectors of (M+1) N^d in the problem.
 */
tsfde_status tsfde_singular_value_estimates(tsfde_problem* prob, int precond, int iters, double* sigma_max,
                                           double* sigma_min, int* iterations, const tsfde_opts* opts,
                                           void* stream);

/*
 * Morozov's discrepancy of a source f (device, N^d): ||v^(M)(f) - mu_eps||_2, with v the solution
 * of the direct problem of §6.1 for f (the first M steps of the forward substitution, block solves
 * to opts->inner_tol).  The largest alpha whose recovered f~ has a discrepancy within tau times the
 * noise norm is Morozov's choice.  residual: host.  Synchronises `stream`.
 */
tsfde_status tsfde_discrepancy(tsfde_problem* prob, const double* f, double* residual, const tsfde_opts* opts,
                               void* stream);

/* Last error message of the calling thread ("" if none). */
const char* tsfde_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TSFDE_H */
