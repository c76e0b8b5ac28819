// Dense-transform block solvers of the §5.1 Remark, for any N: the forward substitution of P with
// every B replaced by Strang's circulant s(B) (S_{n,S}) or by its tau matrix tau(B) (T_{n,S}), and the
// coefficient ratio of each diagonal block frozen at its slice mean sigma_s:
//   s < M:  (sigma_s I + c_t X(B)) y_s = (z_s - gamma1_s sum_{m<s} e_{s-m} y_m) / gamma2_s
//   s = M:  X(B) y_M = (z_M - y_{M-1}) / (c_f gamma2_{M-1}),     X = s or tau.
//
// Strang: a d-level symmetric circulant whose first column c is even along every level is
// diagonalised by the real Hartley transform of size N per level: with H[j][k] = cas(2 pi j k / N),
// cas = cos + sin, H H = N I and
//   s(B) = (H x H) diag(lambda) (H x H) / N^d,
//   lambda[k1][k2] = sum_{l1,l2} c[l1][l2] cos(2 pi l1 k1 / N) cos(2 pi l2 k2 / N)
// (the cos-sin cross terms cancel by the evenness of c).
// tau: tau(B) = (2/(N+1))^d (S x S) diag(lambda) (S x S) with S[j][k] = sin(pi (j+1)(k+1)/(N+1))
// (S S = (N+1)/2 I) and lambda the tau eigenvalues of B.
// Either way every block is solved exactly by two transforms around a diagonal scaling, with no
// inner iterations.  N is arbitrary (it need not give a power-of-two FFT), so each level's transform
// is a dense pass: N multiply-adds per output, the table (Np values, index (j+o)(k+o) mod Np with
// Np = N, o = 0 for cas and Np = 2(N+1), o = 1 for sin) and the workgroup's input rows held in LDS.
// Every pass transforms the fast index of its input and writes its output transposed, so the 2D
// solve is four passes of one kernel and returns to the slice layout [i1][i2].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "grid_sync.hpp"
#include "internal.hpp"
#include "transform_lds.hpp"

namespace tsfde {

constexpr int kCasU = 8;       // unrolled steps of the inner sum

// Where the first pass of a block solve takes its right-hand side from:
//   NEAR: x = w[j] - dg_s[j] sum_{sa <= m < s} e_{s-m} y_m[j], w the far-history slice of step s
//         (dg = e_0 gamma1 / gamma2 with e_0 = 1), i.e. (z_s - gamma1_s sum_{m<s} e_{s-m} y_m) / gamma2_s;
//   LAST: x = (z_M - y_{M-1}) / (c_f gamma2_{M-1});
//   otherwise x = in[j] (scaled by the eigenvalue factor when lam is given).
enum CasSrc : int { SRC_IN = 0, SRC_NEAR = 1, SRC_LAST = 2 };
template <typename T>
struct RhsArgs {
    int mode = SRC_IN;
    int sa = 0, s = 0;
    const T* dg = nullptr;  // dg_s (NEAR); gamma2_{M-1} (LAST)
    const T* y = nullptr;   // the solution so far
    const T* e = nullptr;   // e_0.. (offset into the zero-padded weight table)
    const T* z = nullptr;   // z_M (LAST)
    T cf = T(1);
    long long Nd = 0;
};

template <typename T>
__device__ __forceinline__ T rhs_value(const RhsArgs<T>& ra, const T* __restrict__ in, long long g) {
    if (ra.mode == SRC_NEAR) {
        T h = T(0);
        // at most kHB - 1 near terms; their loads are independent and issued together
#pragma unroll
        for (int t = 1; t < kHB; ++t) {
            const int m = ra.s - t;
            if (m >= ra.sa) h += ra.e[t] * ra.y[(long long)m * ra.Nd + g];
        }
        return in[g] - ra.dg[g] * h;
    }
    if (ra.mode == SRC_LAST) return (ra.z[g] - ra.y[(long long)(ra.s - 1) * ra.Nd + g]) / (ra.cf * ra.dg[g]);
    return in[g];
}

// sum_{j0 <= j < j1} x[j] ct[((j + o)(k + o)) mod Np].  The sum runs in chunks of kCasU: the chunk's
// table indices come from a short VALU chain, so its LDS reads are independent and in flight
// together, and kCasU partial sums break the multiply-add dependence.
template <typename T>
__device__ __forceinline__ T cas_sum(const T* x, const T* ct, int Np, int o, int k, int j0, int j1) {
    T acc[kCasU];
#pragma unroll
    for (int u = 0; u < kCasU; ++u) acc[u] = T(0);
    const int kk = k + o;                                    // < Np
    int idx = (int)(((long long)(j0 + o) * kk) % Np);        // (j + o)(k + o) mod Np
    int j = j0;
    for (; j + kCasU <= j1; j += kCasU) {
        int id[kCasU];
        id[0] = idx;
#pragma unroll
        for (int u = 1; u < kCasU; ++u) {
            const int t = id[u - 1] + kk;
            id[u] = t >= Np ? t - Np : t;
        }
        T cv[kCasU], xv[kCasU];
#pragma unroll
        for (int u = 0; u < kCasU; ++u) {
            cv[u] = ct[id[u]];
            xv[u] = x[j + u];
        }
#pragma unroll
        for (int u = 0; u < kCasU; ++u) acc[u] += xv[u] * cv[u];
        const int t = id[kCasU - 1] + kk;
        idx = t >= Np ? t - Np : t;
    }
    for (; j < j1; ++j) {
        acc[0] += x[j] * ct[idx];
        idx += kk;
        if (idx >= Np) idx -= Np;
    }
    T sum = T(0);
#pragma unroll
    for (int u = 0; u < kCasU; ++u) sum += acc[u];
    return sum;
}

// out[k][r] = sum_j x[r][j] tab[((j + o)(k + o)) mod Np] for r < nrow, k < N, with x[r][j] the
// right-hand side value of point r N + j (rhs_value) times (lam ? scale / (sigma + c lam[r][j]) : 1).
template <typename T>
__global__ __launch_bounds__(256) void cas_pass(const T* __restrict__ in, T* __restrict__ out,
                                                const T* __restrict__ tab, const T* __restrict__ lam, T sigma,
                                                T c, T scale, int N, int Np, int o, int nrow, RhsArgs<T> ra) {
    extern __shared__ double cas_lds_raw[];
    T* ct = reinterpret_cast<T*>(cas_lds_raw);  // [Np]
    T* xs = ct + Np;                             // [nr][N]
    __shared__ T part[4][kCasK];                 // partial sums of a single row (d = 1)
    const int r0 = blockIdx.y * kCasRows;
    const int nr = min(kCasRows, nrow - r0);
    for (int i = threadIdx.x; i < Np; i += blockDim.x) ct[i] = tab[i];
    const long long base = (long long)r0 * N;
    for (int i = threadIdx.x; i < nr * N; i += blockDim.x) {
        T v = rhs_value(ra, in, base + i);
        if (lam) v *= scale / (sigma + c * lam[base + i]);
        xs[i] = v;
    }
    __syncthreads();
    const int k = blockIdx.x * kCasK + (threadIdx.x & (kCasK - 1));
    const int w = threadIdx.x / kCasK;
    if (nrow == 1) {
        // a single row (d = 1): the four waves split the sum over j and add their partial sums
        const int span = (N + 3) / 4;
        const int j0 = min(N, w * span), j1 = min(N, j0 + span);
        part[w][threadIdx.x & (kCasK - 1)] = k < N ? cas_sum(xs, ct, Np, o, k, j0, j1) : T(0);
        __syncthreads();
        if (w == 0 && k < N) {
            const int l = threadIdx.x;
            out[k] = (part[0][l] + part[1][l]) + (part[2][l] + part[3][l]);
        }
        return;
    }
    const int r = w;  // one row per wave
    if (k >= N || r >= nr) return;
    const T sum = cas_sum(xs + r * N, ct, Np, o, k, 0, N);
    out[(long long)k * nrow + r0 + r] = sum;
}

// the transform of a block solver: its table, period and index offset, eigenvalues and the scale
// of the inverse (1 / N^d for Hartley, (2/(N+1))^d for sine)
template <typename T>
struct DenseXf {
    const T* tab;
    const T* lam;   // eigenvalues [k1][k2]
    const T* lamT;  // transposed [k2][k1]
    int Np, o;
    T inv;
};

bool strang_supported(const Problem& P) { return dense_blocks_fit(P.d, P.N, P.N); }
bool tau_dense_supported(const Problem& P) { return dense_blocks_fit(P.d, P.N, 2 * (P.N + 1)); }

template <typename T>
static void cas_launch(const T* in, T* out, const DenseXf<T>& X, const T* lam, T sigma, T c, T scale, int N,
                       int nrow, hipStream_t st, const RhsArgs<T>& ra = RhsArgs<T>()) {
    const dim3 grid((unsigned)((N + kCasK - 1) / kCasK), (unsigned)((nrow + kCasRows - 1) / kCasRows));
    const size_t lds = pass_dyn_lds(N, X.Np, nrow, sizeof(T));
    hipLaunchKernelGGL(cas_pass<T>, grid, dim3(256), lds, st, in, out, X.tab, lam, sigma, c, scale, N, X.Np, X.o,
                       nrow, ra);
    TSFDE_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Persistent form: one launch per segment of kHB steps (after far_history), the passes of a step
// separated by device-wide barriers, workgroups of 16 waves.
// 2D: a workgroup owns a block of kCasRows rows; wave w handles row w % 4 and the outputs of chunk
// group w / 4 (outputs k = 64 (w / 4) + lane + 256 t):
//   [P1]  rows i1 of the step's right-hand side (near history added) -> t1[k2][i1]
//   [P23] rows k2 of t1: transform over i1, scale by inv / (sigma + c lam[k1][k2]), transform back
//         -> t2[m1][k2]
//   [P4]  rows m1 of t2: transform over k2 -> y_s[m1][m2], then at once [P1] of step s + 1 on the same
//         rows (its near history is pointwise in space, so it reads only rows this workgroup wrote)
// so a step costs two barriers.
// 1D: the outputs of a transform are dealt out in chunks of 64 over the workgroups, the 16 waves of a
// workgroup splitting the sum over j:
//   [P1]  the right-hand side row (t2) -> t1
//   [P2]  t1 scaled -> y_s, then the right-hand side of step s + 1 at the same points (pointwise
//         near history) -> t2
// again two barriers per step.
// ---------------------------------------------------------------------------
constexpr int kSegWaves = 16;
constexpr int kSegThreads = 64 * kSegWaves;

template <typename T>
struct DenseSegArgs {
    int d, N, M, Np, o;
    long long Nd;
    const T* tab;   // [Np]
    const T* lamT;  // [Nd] eigenvalues transposed, lamT[k2][k1] (1D: lam[k])
    const double* sigma;  // [M]
    T ct, cf, inv;
    const T* z;
    T* y;
    const T* hacc;  // [kHB][Nd] far-history right-hand sides of the segment's steps
    const T* dg;    // [M][Nd]
    const T* g2;    // [M][Nd]
    const T* e;     // e_0.. (epad + kEpad)
    T* t1;
    T* t2;
    unsigned* bar;
    unsigned long long bar_ticks;
};

// right-hand side of step s at point g: near history on top of the far-history slice, or the last row
template <typename T>
__device__ __forceinline__ T seg_rhs(const DenseSegArgs<T>& a, int sa, int s, long long g) {
    if (s == a.M)
        return (a.z[(long long)a.M * a.Nd + g] - a.y[(long long)(a.M - 1) * a.Nd + g]) /
               (a.cf * a.g2[(long long)(a.M - 1) * a.Nd + g]);
    T h = T(0);
#pragma unroll
    for (int t = 1; t < kHB; ++t) {
        const int m = s - t;
        if (m >= sa) h += a.e[t] * a.y[(long long)m * a.Nd + g];
    }
    return a.hacc[(long long)(s - sa) * a.Nd + g] - a.dg[(long long)s * a.Nd + g] * h;
}

template <typename T>
__global__ __launch_bounds__(kSegThreads) void dense_segment(DenseSegArgs<T> a, int sa, int sb) {
    extern __shared__ double seg_lds_raw[];
    T* ct = reinterpret_cast<T*>(seg_lds_raw);  // [Np]
    T* xs = ct + a.Np;                            // [kCasRows][N] inputs of a pass (1D: [N])
    T* ys = xs + (size_t)kCasRows * a.N;          // [kCasRows][N] forward results of P23 (2D)
    __shared__ T part[kSegWaves][kCasK];
    const int N = a.N, Np = a.Np, o = a.o;
    const int lane = threadIdx.x & (kCasK - 1);
    const int w = threadIdx.x / kCasK;
    for (int i = threadIdx.x; i < Np; i += blockDim.x) ct[i] = a.tab[i];
    unsigned epoch = 0;
    const int last = sb - 1;
    if (a.d == 2) {
        const int nrb = (N + kCasRows - 1) / kCasRows;
        const int r = w % kCasRows;                 // this wave's row of the block
        const int kc0 = (w / kCasRows) * kCasK;     // its first output, then every 256
        constexpr int kStep = kCasK * (kSegWaves / kCasRows);
        auto p1 = [&](int s, int rb) {
            const int r0 = rb * kCasRows;
            const int nr = min(kCasRows, N - r0);
            for (int i = threadIdx.x; i < nr * N; i += blockDim.x) xs[i] = seg_rhs(a, sa, s, (long long)r0 * N + i);
            __syncthreads();
            if (r < nr)
                for (int k = kc0 + lane; k < N; k += kStep) a.t1[(long long)k * N + r0 + r] = cas_sum(xs + r * N, ct, Np, o, k, 0, N);
            __syncthreads();
        };
        for (int rb = blockIdx.x; rb < nrb; rb += gridDim.x) p1(sa, rb);
        for (int s = sa; s <= last; ++s) {
            grid_barrier(a.bar, a.bar_ticks, epoch);
            // [P23] rows k2 of t1 -> t2 columns
            const T sig = s < a.M ? T(a.sigma[s]) : T(0);
            const T c = s < a.M ? a.ct : T(1);
            for (int rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
                const int k0 = rb * kCasRows;
                const int nr = min(kCasRows, N - k0);
                for (int i = threadIdx.x; i < nr * N; i += blockDim.x) xs[i] = a.t1[(long long)k0 * N + i];
                __syncthreads();
                if (r < nr) {
                    const T* lrow = a.lamT + (long long)(k0 + r) * N;
                    for (int k1 = kc0 + lane; k1 < N; k1 += kStep)
                        ys[r * N + k1] = cas_sum(xs + r * N, ct, Np, o, k1, 0, N) * a.inv / (sig + c * lrow[k1]);
                }
                __syncthreads();
                if (r < nr)
                    for (int m1 = kc0 + lane; m1 < N; m1 += kStep)
                        a.t2[(long long)m1 * N + k0 + r] = cas_sum(ys + r * N, ct, Np, o, m1, 0, N);
                __syncthreads();
            }
            grid_barrier(a.bar, a.bar_ticks, epoch);
            // [P4] rows m1 of t2 -> y_s rows, then [P1] of the next step on the same rows
            T* yst = a.y + (long long)s * a.Nd;
            for (int rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
                const int m0 = rb * kCasRows;
                const int nr = min(kCasRows, N - m0);
                for (int i = threadIdx.x; i < nr * N; i += blockDim.x) xs[i] = a.t2[(long long)m0 * N + i];
                __syncthreads();
                if (r < nr)
                    for (int m2 = kc0 + lane; m2 < N; m2 += kStep)
                        yst[(long long)(m0 + r) * N + m2] = cas_sum(xs + r * N, ct, Np, o, m2, 0, N);
                __syncthreads();
                if (s < last) p1(s + 1, rb);
            }
        }
        return;
    }
    // d = 1
    const int nkc = (N + kCasK - 1) / kCasK;
    const int span = (N + kSegWaves - 1) / kSegWaves;
    const int j0 = min(N, w * span), j1 = min(N, j0 + span);
    // one chunk of outputs: sum over the waves' parts of x . table
    auto chunk = [&](const T* x, int k) -> T {
        part[w][lane] = k < N ? cas_sum(x, ct, Np, o, k, j0, j1) : T(0);
        __syncthreads();
        T sum = T(0);
        if (w == 0) {
#pragma unroll
            for (int q = 0; q < kSegWaves; ++q) sum += part[q][lane];
        }
        __syncthreads();
        return sum;
    };
    // the right-hand side of the first step at this workgroup's chunks
    for (int kc = blockIdx.x; kc < nkc; kc += gridDim.x)
        for (int m = kc * kCasK + (int)threadIdx.x; m < min(N, (kc + 1) * kCasK); m += blockDim.x) a.t2[m] = seg_rhs(a, sa, sa, m);
    for (int s = sa; s <= last; ++s) {
        grid_barrier(a.bar, a.bar_ticks, epoch);
        // [P1] the right-hand side row -> t1
        for (int i = threadIdx.x; i < N; i += blockDim.x) xs[i] = a.t2[i];
        __syncthreads();
        for (int kc = blockIdx.x; kc < nkc; kc += gridDim.x) {
            const int k = kc * kCasK + lane;
            const T v = chunk(xs, k);
            if (w == 0 && k < N) a.t1[k] = v;
        }
        grid_barrier(a.bar, a.bar_ticks, epoch);
        // [P2] scaled t1 -> y_s; the next step's right-hand side at the same points
        const T sig = s < a.M ? T(a.sigma[s]) : T(0);
        const T c = s < a.M ? a.ct : T(1);
        for (int i = threadIdx.x; i < N; i += blockDim.x) xs[i] = a.t1[i] * a.inv / (sig + c * a.lamT[i]);
        __syncthreads();
        T* yst = a.y + (long long)s * a.Nd;
        for (int kc = blockIdx.x; kc < nkc; kc += gridDim.x) {
            const int m = kc * kCasK + lane;
            const T v = chunk(xs, m);
            if (w == 0 && m < N) yst[m] = v;
            __syncthreads();  // the chunk's y_s values written before the next right-hand side reads them
            if (s < last)
                for (int q = kc * kCasK + (int)threadIdx.x; q < min(N, (kc + 1) * kCasK); q += blockDim.x)
                    a.t2[q] = seg_rhs(a, sa, s + 1, q);
        }
    }
}

// dynamic LDS of the persistent segment kernel: the table, the inputs and (2D) the forward results
static size_t dense_seg_lds(int d, int N, int Np, size_t elem) {
    return ((size_t)Np + (d == 2 ? 2 * (size_t)kCasRows * (size_t)N : (size_t)N)) * elem;
}

// ---------------------------------------------------------------------------
// 2D FP64 passes on the matrix cores.  A pass is the product D = C X^T, C[k][j] the transform's table
// matrix (tab[((j+o)(k+o)) mod Np], zero past N, stored Kp x Kp with Kp = N rounded up to 16) and
// X[r][j] its input rows:  D[k][r] = sum_j C[k][j] X[r][j], written row-major [k][r] (the transposed
// layout the next pass reads).  v_mfma_f64_16x16x4f64 takes A[i][q] from lane i + 16 q, B[q][jj] from
// lane jj + 16 q, and leaves D[i][jj] in lane jj + 16 (i % 4), value i / 4.  A workgroup of four waves
// computes one 16 x 16 tile of D, each wave a quarter of the sum over j; inside a wave the lanes of
// group q = lane / 16 take a contiguous run of that quarter (the order of a sum's terms is free), so
// every lane reads whole cache lines.  The quarters are added in LDS.
// The input is read plainly or formed as the last row's right-hand side (z_M - y_{M-1}) /
// (c_f gamma2_{M-1}).  The second pass of a step stores its output
// scaled by the eigenvalue factor (once per value, where scaling the third pass's input would repeat
// the division in every tile that reads it); the last pass writes y_s and, at the same points, the
// right-hand side of step s + 1 (its near history is pointwise in space), so the next step's first
// pass reads it plainly.
// ---------------------------------------------------------------------------
enum MfmaIn : int { MIN_PLAIN = 0, MIN_LAST = 2 };
// what a pass does with its output besides storing it: nothing, the eigenvalue scaling (then stored
// scaled), or forming the next step's right-hand side
enum MfmaEpi : int { EPI_NONE = 0, EPI_SCALE = 1, EPI_NEXT = 2 };

struct MfmaPassArgs {
    const double* in;
    double* out;
    const double* Cm;  // [Kp][Kp]
    int Kp, N;
    // EPI_SCALE
    const double* lam;  // [k1][k2], the output index of the scaled pass
    double sigma, c, scale;
    // MIN_LAST, and the SRC_LAST right-hand side of the epilogue
    const double* z;   // z_M
    const double* yl;  // y_{M-1}
    const double* g2;  // gamma2_{M-1}
    double cf;
    // epilogue (last pass of step s): rhs of step s + 1 = s1
    int next;  // 0: none, SRC_NEAR, SRC_LAST
    int sa, s1;
    long long Nd;
    const double* hacc;  // w_{s1}, the far-history slice (SRC_NEAR)
    const double* dg;    // dg_{s1} (SRC_NEAR)
    const double* y;     // the solution so far
    const double* e;     // e_0..
    double* rhs;
};

typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaRun = 4;  // unrolled MFMA steps of a lane group's run

template <int IN>
__device__ __forceinline__ double mfma_in(const MfmaPassArgs& a, int r, int j) {
    if (r >= a.N || j >= a.N) return 0.0;
    const long long g = (long long)r * a.N + j;
    if (IN == MIN_LAST) return (a.z[g] - a.yl[g]) / (a.cf * a.g2[g]);
    return a.in[g];
}

template <int IN, int EPI>
__global__ __launch_bounds__(256) void mfma_pass(MfmaPassArgs a) {
    __shared__ double red[4][256];
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int k0 = blockIdx.x * 16, r0 = blockIdx.y * 16;
    const int run = a.Kp >> 4;                       // a lane group's share of the wave's quarter
    const int jb = (w * 4 + (l >> 4)) * run;         // its first j
    const double* crow = a.Cm + (long long)(k0 + (l & 15)) * a.Kp + jb;
    const int r = r0 + (l & 15);
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    int t = 0;
    for (; t + kMfmaRun <= run; t += kMfmaRun) {
        double av[kMfmaRun], bv[kMfmaRun];
#pragma unroll
        for (int u = 0; u < kMfmaRun; ++u) {
            av[u] = crow[t + u];
            bv[u] = mfma_in<IN>(a, r, jb + t + u);
        }
#pragma unroll
        for (int u = 0; u < kMfmaRun; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    for (; t < run; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(crow[t], mfma_in<IN>(a, r, jb + t), acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) red[v][w * 64 + l] = acc[v];
    __syncthreads();
    // wave w finishes value w of every lane: D[k][r] with k = k0 + l / 16 + 4 w
    const double d = (red[w][l] + red[w][64 + l]) + (red[w][128 + l] + red[w][192 + l]);
    const int k = k0 + (l >> 4) + 4 * w;
    if (k >= a.N || r >= a.N) return;
    const long long g = (long long)k * a.N + r;
    if (EPI == EPI_SCALE) {  // the eigenvalue step on this pass's output [k1][k2]
        a.out[g] = d * (a.scale / (a.sigma + a.c * a.lam[g]));
        return;
    }
    a.out[g] = d;
    if (EPI != EPI_NEXT) return;
    if (a.next == SRC_NEAR) {
        // rhs_{s1} = w_{s1} - dg_{s1} sum_{sa <= m < s1} e_{s1-m} y_m, with y_{s1-1} = d
        double h = a.e[1] * d;
#pragma unroll
        for (int q = 2; q < kHB; ++q) {
            const int m = a.s1 - q;
            if (m >= a.sa) h += a.e[q] * a.y[(long long)m * a.Nd + g];
        }
        a.rhs[g] = a.hacc[g] - a.dg[g] * h;
    } else if (a.next == SRC_LAST) {
        a.rhs[g] = (a.z[g] - d) / (a.cf * a.g2[g]);
    }
}

template <int IN, int EPI>
static void mfma_launch(const MfmaPassArgs& a, hipStream_t st) {
    const dim3 grid((unsigned)(a.Kp / 16), (unsigned)(a.Kp / 16));
    hipLaunchKernelGGL((mfma_pass<IN, EPI>), grid, dim3(256), 0, st, a);
    TSFDE_HIP(hipGetLastError());
}

template <typename T>
static T* table(Problem& P, bool tau);
template <>
double* table<double>(Problem& P, bool tau) { return tau ? P.taud64 : P.strang64; }
template <>
float* table<float>(Problem& P, bool tau) { return tau ? P.taud32 : P.strang32; }

// Uploads [table][eigenvalues] in FP64 and FP32, and (once) the far-history slices of a block of steps.
static void upload_tables(Problem& P, const std::vector<double>& tab, const std::vector<double>& lam, double*& d64,
                          float*& d32) {
    std::vector<double> t(tab);
    t.insert(t.end(), lam.begin(), lam.end());
    // the eigenvalues again, transposed (lamT[k2][k1]), for the persistent solver's column pass
    const int N = P.N;
    if (P.d == 2) {
        for (int k2 = 0; k2 < N; ++k2)
            for (int k1 = 0; k1 < N; ++k1) t.push_back(lam[(size_t)k1 * N + k2]);
    } else {
        t.insert(t.end(), lam.begin(), lam.end());
    }
    std::vector<float> t32(t.begin(), t.end());
    if (P.d == 2) {
        // the table matrix C[k][j] = tab[((j + o)(k + o)) mod Np] (FP64 only), Kp x Kp, zero past N
        const int Kp = (N + 15) / 16 * 16;
        const long long Np = (long long)tab.size();
        const int o = Np == N ? 0 : 1;
        const size_t base = t.size();
        t.resize(base + (size_t)Kp * Kp, 0.0);
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j) t[base + (size_t)k * Kp + j] = tab[((long long)(j + o) * (k + o)) % Np];
    }
    dev_alloc(P, d64, t.size());
    dev_alloc(P, d32, t32.size());
    TSFDE_HIP(hipMemcpy(d64, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice));
    TSFDE_HIP(hipMemcpy(d32, t32.data(), sizeof(float) * t32.size(), hipMemcpyHostToDevice));
    if (!P.strang_hist) dev_alloc(P, P.strang_hist, (size_t)kHB * P.Nd);
}

// The cas table and the eigenvalues of s(B), computed on first use: [N] cas(2 pi m / N), then
// [Nd] lambda (2D: [k1][k2], k2 the frequency of the fast index).
void ensure_strang(Problem& P) {
    if (P.strang64) return;
    std::vector<double> cas, lam;
    const double lmin = strang_tables(P, cas, lam);
    upload_tables(P, cas, lam, P.strang64, P.strang32);
    P.strang_min = lmin;
}

// The sine table and the tau eigenvalues of B for the dense T_{n,S} blocks: [2(N+1)] sin(pi m/(N+1)),
// then [Nd] lambda ([k1][k2]).
void ensure_tau_dense(Problem& P) {
    if (P.taud64) return;
    std::vector<double> tab, lam;
    const double lmin = tau_dense_tables(P, tab, lam);
    upload_tables(P, tab, lam, P.taud64, P.taud32);
    P.taud_min = lmin;
}

// The steps run in blocks of kHB: one bandwidth-bound kernel folds the history of all earlier blocks
// into the block's right-hand sides, and each step's first transform pass adds the (< kHB) near terms
// while loading its rows.
// The persistent form of the block solves: far_history and one dense_segment launch per segment of
// kHB steps, the grid holding its CU slots until the host has seen the last segment finish.
template <typename T>
static void dense_persistent(Problem& P, const Dev<T>& D, const T* z, T* y, const DenseXf<T>& X, T* t1, T* t2,
                             T* hist, int last, size_t lds, hipStream_t st) {
    if (!P.dense_bar) dev_alloc(P, P.dense_bar, 16);
    int dev = 0, ncu = 0, per_cu = 0;
    TSFDE_HIP(hipGetDevice(&dev));
    TSFDE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    TSFDE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dense_segment<T>, kSegThreads, lds));
    if (per_cu < 1) throw HipError{hipErrorInvalidConfiguration, "dense block solver: a workgroup does not fit a CU"};
    ResidencyBudget& pool = residency_budget(dev, ncu);
    const int work = P.d == 2 ? (P.N + kCasRows - 1) / kCasRows : (P.N + kCasK - 1) / kCasK;
    int cap = std::min(per_cu * ncu, residency_max_grid(pool.total(), kXcds));
    if (shared_launch()) cap = std::min(cap, std::max(1, ncu / kMaxInflight));
    const int grid = std::max(1, std::min(work, cap));
    ResidencyTicket ticket;
    ticket.hold(&pool, residency_slots(grid, kXcds));
    DenseSegArgs<T> a{};
    a.d = P.d;
    a.N = P.N;
    a.M = P.M;
    a.Np = X.Np;
    a.o = X.o;
    a.Nd = P.Nd;
    a.tab = X.tab;
    a.lamT = X.lamT;
    a.sigma = P.d_sigma;
    a.ct = T(P.ct);
    a.cf = T(P.cf);
    a.inv = X.inv;
    a.z = z;
    a.y = y;
    a.hacc = hist;
    a.dg = D.dg;
    a.g2 = D.gamma2;
    a.e = D.epad + kEpad;
    a.t1 = t1;
    a.t2 = t2;
    a.bar = P.dense_bar;
    a.bar_ticks = barrier_ticks(dev);
    launch_fill(reinterpret_cast<float*>(P.dense_bar) + 1, 1, 0.0f, st);  // clear the abort word
    for (int sa = 0; sa <= last; sa += kHB) {
        const int cnt = std::min(kHB, P.M - sa);
        if (cnt > 0) launch_far_history<T>(P, D, y, hist, z, sa, cnt, st);
        int sa_ = sa, sb_ = std::min(sa + kHB, last + 1);
        launch_fill(reinterpret_cast<float*>(P.dense_bar), 1, 0.0f, st);  // zero the barrier counter
        void* args[] = {&a, &sa_, &sb_};
        TSFDE_HIP(hipLaunchKernel((void*)dense_segment<T>, dim3(grid), dim3(kSegThreads), args, lds, st));
    }
    unsigned* abort_h = reinterpret_cast<unsigned*>(P.host_scalars + 58);
    TSFDE_HIP(hipMemcpyAsync(abort_h, P.dense_bar + 1, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    TSFDE_HIP(hipStreamSynchronize(st));
    if (*abort_h != 0u)
        throw HipError{hipErrorLaunchTimeOut, "dense block solver: a device-wide barrier wait timed out"};
}

// The 2D FP64 block solves on the matrix cores: per step four mfma_pass launches,
//   rhs [i1][i2] -> t1 [k2][i1] -> t2 [k1][k2] -> (scaled) t1 [m2][k1] -> y_s [m1][m2],
// the last one also writing the right-hand side of step s + 1 into t2 (free by then).  The first
// step of a block of kHB steps reads its right-hand side from the far-history slice (or forms the
// last row's).
static void dense_mfma(Problem& P, const Dev<double>& D, const double* z, double* y, const DenseXf<double>& X,
                       double* t1, double* t2, double* hist, int last, hipStream_t st) {
    const int N = P.N;
    const long long Nd = P.Nd;
    MfmaPassArgs a{};
    a.N = N;
    a.Kp = (N + 15) / 16 * 16;
    a.Cm = X.lamT + Nd;
    a.lam = X.lam;
    a.z = z + (long long)P.M * Nd;
    a.yl = y + (long long)(P.M - 1) * Nd;
    a.g2 = D.gamma2 + (long long)(P.M - 1) * Nd;
    a.cf = P.cf;
    a.Nd = Nd;
    a.y = y;
    a.e = D.epad + kEpad;
    a.rhs = t2;
    for (int sa = 0; sa <= last; sa += kHB) {
        const int cnt = std::min(kHB, P.M - sa);
        if (cnt > 0) launch_far_history<double>(P, D, y, hist, z, sa, cnt, st);
        const int se = std::min(sa + kHB - 1, last);
        a.sa = sa;
        for (int s = sa; s <= se; ++s) {
            MfmaPassArgs p = a;
            p.out = t1;
            if (s > sa) {
                p.in = t2;
                mfma_launch<MIN_PLAIN, EPI_NONE>(p, st);
            } else if (s < P.M) {
                p.in = hist;
                mfma_launch<MIN_PLAIN, EPI_NONE>(p, st);
            } else {
                mfma_launch<MIN_LAST, EPI_NONE>(p, st);
            }
            // [k2][i1] -> [k1][k2], each value scaled once by scale / (sigma + c lam[k1][k2])
            p.in = t1;
            p.out = t2;
            p.sigma = s < P.M ? P.sigma[s] : 0.0;
            p.c = s < P.M ? P.ct : 1.0;
            p.scale = X.inv;
            mfma_launch<MIN_PLAIN, EPI_SCALE>(p, st);
            p.in = t2;
            p.out = t1;
            mfma_launch<MIN_PLAIN, EPI_NONE>(p, st);
            p.in = t1;
            p.out = y + (long long)s * Nd;
            p.s1 = s + 1;
            p.next = s + 1 > se ? 0 : (s + 1 < P.M ? SRC_NEAR : SRC_LAST);
            p.hacc = hist + (long long)(s + 1 - sa) * Nd;
            p.dg = s + 1 < P.M ? D.dg + (long long)(s + 1) * Nd : nullptr;
            mfma_launch<MIN_PLAIN, EPI_NEXT>(p, st);
        }
    }
}

template <typename T>
void pinv_dense_blocks(Problem& P, const Dev<T>& D, const T* z, T* y, bool last_block, bool tau, hipStream_t st) {
    if (tau) ensure_tau_dense(P);
    else ensure_strang(P);
    const long long Nd = P.Nd;
    const int N = P.N;
    DenseXf<T> X;
    X.tab = table<T>(P, tau);
    X.Np = tau ? 2 * (N + 1) : N;
    X.o = tau ? 1 : 0;
    X.lam = X.tab + X.Np;
    X.lamT = X.lam + Nd;
    X.inv = tau ? T(std::pow(2.0 / (N + 1), P.d)) : T(1.0 / (double)Nd);  // S S = (N+1)/2 I;  H H = N I
    const T* lam = X.lam;
    const int nrow = P.d == 2 ? N : 1;
    T* t1 = D.pcg + 5 * Nd;
    T* t2 = D.pcg + 6 * Nd;
    T* hist = reinterpret_cast<T*>(P.strang_hist);
    const T inv = X.inv;
    const int last = last_block ? P.M : P.M - 1;
    const size_t seg_lds = dense_seg_lds(P.d, N, X.Np, sizeof(T));
    // the persistent form is the faster one for a single row (d = 1: 52 against 91 ms at N = 4095,
    // M = 1024); in 2D the one-launch-per-pass form spreads each pass over more CUs (13.4 against
    // 20.6 ms at N = 255, M = 256: the passes are bound by the LDS table reads of the sums).
    // TSFDE_DENSE_PERSISTENT=1 / 0 forces either.
    const char* pe = std::getenv("TSFDE_DENSE_PERSISTENT");
    const bool persistent = pe ? std::atoi(pe) != 0 : P.d == 1;
    if (persistent) {
        if (seg_lds + sizeof(T) * kSegWaves * kCasK <= kPassLdsBytes) {
            dense_persistent<T>(P, D, z, y, X, t1, t2, hist, last, seg_lds, st);
            return;
        }
    }
    if constexpr (std::is_same<T, double>::value) {
        // 2D in FP64: the passes on the matrix cores (TSFDE_DENSE_MFMA=0 selects the LDS-table passes)
        const char* me = std::getenv("TSFDE_DENSE_MFMA");
        if (P.d == 2 && (!me || std::atoi(me) != 0)) {
            dense_mfma(P, D, z, y, X, t1, t2, hist, last, st);
            return;
        }
    }
    for (int sa = 0; sa <= last; sa += kHB) {
        const int cnt = std::min(kHB, P.M - sa);
        if (cnt > 0) launch_far_history<T>(P, D, y, hist, z, sa, cnt, st);
        for (int s = sa; s <= std::min(sa + kHB - 1, last); ++s) {
            RhsArgs<T> ra;
            ra.sa = sa;
            ra.s = s;
            ra.y = y;
            ra.e = D.epad + kEpad;
            ra.Nd = Nd;
            const T* in = nullptr;
            if (s < P.M) {
                ra.mode = SRC_NEAR;
                ra.dg = D.dg + (long long)s * Nd;
                in = hist + (long long)(s - sa) * Nd;
            } else {
                ra.mode = SRC_LAST;
                ra.dg = D.gamma2 + (long long)(P.M - 1) * Nd;
                ra.z = z + (long long)P.M * Nd;
                ra.cf = T(P.cf);
            }
            const T sigma = (s < P.M) ? T(P.sigma[s]) : T(0);
            const T c = (s < P.M) ? T(P.ct) : T(1);
            T* ys = y + (long long)s * Nd;
            cas_launch<T>(in, t1, X, nullptr, T(0), T(0), T(1), N, nrow, st, ra);  // [i1][i2] -> [k2][i1]
            if (P.d == 1) {
                cas_launch<T>(t1, ys, X, lam, sigma, c, inv, N, 1, st);
            } else {
                cas_launch<T>(t1, t2, X, nullptr, T(0), T(0), T(1), N, N, st);  // -> [k1][k2]
                cas_launch<T>(t2, t1, X, lam, sigma, c, inv, N, N, st);         // scaled, -> [m2][k1]
                cas_launch<T>(t1, ys, X, nullptr, T(0), T(0), T(1), N, N, st);  // -> [m1][m2]
            }
        }
    }
}

template <typename T>
void pinv_strang(Problem& P, const Dev<T>& D, const T* z, T* y, bool last_block, hipStream_t st) {
    pinv_dense_blocks<T>(P, D, z, y, last_block, false, st);
}

template <typename T>
void pinv_tau_dense(Problem& P, const Dev<T>& D, const T* z, T* y, bool last_block, hipStream_t st) {
    pinv_dense_blocks<T>(P, D, z, y, last_block, true, st);
}

template void pinv_strang<double>(Problem&, const Dev<double>&, const double*, double*, bool, hipStream_t);
template void pinv_strang<float>(Problem&, const Dev<float>&, const float*, float*, bool, hipStream_t);
template void pinv_tau_dense<double>(Problem&, const Dev<double>&, const double*, double*, bool, hipStream_t);
template void pinv_tau_dense<float>(Problem&, const Dev<float>&, const float*, float*, bool, hipStream_t);

}  // namespace tsfde
