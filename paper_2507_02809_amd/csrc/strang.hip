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
    const T* lam;
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
    std::vector<float> t32(t.begin(), t.end());
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
    X.inv = tau ? T(std::pow(2.0 / (N + 1), P.d)) : T(1.0 / (double)Nd);  // S S = (N+1)/2 I;  H H = N I
    const T* lam = X.lam;
    const int nrow = P.d == 2 ? N : 1;
    T* t1 = D.pcg + 5 * Nd;
    T* t2 = D.pcg + 6 * Nd;
    T* hist = reinterpret_cast<T*>(P.strang_hist);
    const T inv = X.inv;
    const int last = last_block ? P.M : P.M - 1;
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
