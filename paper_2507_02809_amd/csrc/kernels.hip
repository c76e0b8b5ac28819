// Streaming kernels: the time-history part of A y (§5 matvec step 1(a)), the history
// right-hand side of each forward-substitution step for P (§5.1), CG vector updates,
// Arnoldi (classical Gram-Schmidt) reductions and small vector helpers.
#include <algorithm>

#include <type_traits>

#include "internal.hpp"

namespace tsfde {

// ---------------------------------------------------------------------------
// z^(s) = gamma1^(s) .* sum_{m=1}^{s} e_{s-m} y^(m) - eta q^(s) y^(M+1),  s = 1..M
// (0-based here: s = 0..M-1, y[M] is f~).
//
// One workgroup = 64 spatial points (one per lane) x 16 NW output steps (16 per wave, NW waves);
// every input step is read once per 16 NW outputs.  The input steps are staged through
// LDS 16 at a time, double-buffered: the loads of the next 16 steps are in flight while the
// current ones are used, and one barrier per stage suffices.  e_{s-m} is wave-uniform, so the
// weights come from the scalar cache; epad holds kEpad zeros before e_0 so that e_{s-m} with
// m > s reads a zero.  A wave skips the stages that lie entirely after its outputs.
// ---------------------------------------------------------------------------
constexpr int kHistStage = 16;  // input steps per stage (and output steps per wave)

template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void history_matvec(const T* __restrict__ y, T* __restrict__ z,
                                                          const T* __restrict__ g1, const T* __restrict__ epad,
                                                          const T* __restrict__ q, T eta, long long Nd, int M) {
    constexpr int NT = 64 * NW;                        // threads
    constexpr int PER = kHistStage * 64 / NT;          // staged values per thread and stage
    static_assert(PER >= 1 && PER * NT == kHistStage * 64, "one stage is 16 steps x 64 points");
    __shared__ T tile[2][kHistStage][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long j = (long long)blockIdx.x * 64 + lane;
    const int s0 = blockIdx.y * (kHistStage * NW);
    const int sw = s0 + wave * kHistStage;
    const int s_end = min(s0 + kHistStage * NW, M);  // inputs m < s_end contribute
    const int nstage = (s_end + kHistStage - 1) / kHistStage;
    T acc[kHistStage];
#pragma unroll
    for (int i = 0; i < kHistStage; ++i) acc[i] = T(0);
    // thread t stages rows mm = t / 64 + (NT / 64) r of a stage, point column lane
    T pre[PER];
    auto stage_load = [&](int m0) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int m = m0 + (int)(threadIdx.x >> 6) + NW * r;
            pre[r] = (m < s_end && j < Nd) ? y[(long long)m * Nd + j] : T(0);
        }
    };
    stage_load(0);
    for (int t = 0; t < nstage; ++t) {
        const int buf = t & 1;
#pragma unroll
        for (int r = 0; r < PER; ++r) tile[buf][(threadIdx.x >> 6) + NW * r][lane] = pre[r];
        __syncthreads();  // stage t visible; every wave is past stage t - 1, so buffer buf ^ 1 is free
        const int m0 = t * kHistStage;
        if (t + 1 < nstage) stage_load(m0 + kHistStage);
        if (sw < M && m0 <= sw + kHistStage - 1) {  // (sw < M keeps the weight reads inside epad)
            const T* ew = epad + kEpad + sw - m0;
#pragma unroll
            for (int mm = 0; mm < kHistStage; ++mm) {
                const T yv = tile[buf][mm][lane];
#pragma unroll
                for (int i = 0; i < kHistStage; ++i) acc[i] += ew[i - mm] * yv;
            }
        }
    }
    if (j < Nd) {
        const T f = y[(long long)M * Nd + j];
#pragma unroll
        for (int i = 0; i < kHistStage; ++i) {
            const int s = sw + i;
            if (s < M) z[(long long)s * Nd + j] = g1[(long long)s * Nd + j] * acc[i] - eta * q[s] * f;
        }
    }
}

template <typename T>
void launch_history_matvec(const Problem& P, const Dev<T>& D, const T* y, T* z, hipStream_t s) {
    // 4 waves (64 output steps per workgroup): measured at c3 as fast as 8 waves and faster than 16
    // (FP64 134 us against 135 and 181 us), with the most workgroups for short histories
    constexpr int NW = 4;
    dim3 grid((unsigned)((P.Nd + 63) / 64), (unsigned)((P.M + NW * kHistStage - 1) / (NW * kHistStage)));
    hipLaunchKernelGGL((history_matvec<T, NW>), grid, dim3(64 * NW), 0, s, y, z, D.gamma1, D.epad, D.q, T(P.eta),
                       P.Nd, P.M);
    TSFDE_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// right-hand side of forward-substitution step s (0-based):
//   s < M : rhs = (z^(s) - gamma1^(s) .* sum_{m<s} e_{s-m} y^(m)) ./ gamma2^(s)
//   s = M : rhs = (z^(M) - y^(M-1)) ./ (cf gamma2^(M-1))          (last block row)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void step_rhs(const T* __restrict__ z, const T* __restrict__ y, const T* __restrict__ g1,
                         const T* __restrict__ g2, const T* __restrict__ epad, int s, int M, long long Nd,
                         T cf, T* __restrict__ rhs) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Nd) return;
    if (s == M) {
        rhs[j] = (z[(long long)M * Nd + j] - y[(long long)(M - 1) * Nd + j]) / (cf * g2[(long long)(M - 1) * Nd + j]);
        return;
    }
    T h = T(0);
    const T* e = epad + kEpad;
    for (int m = 0; m < s; ++m) h += e[s - m] * y[(long long)m * Nd + j];
    const long long o = (long long)s * Nd + j;
    rhs[j] = (z[o] - g1[o] * h) / g2[o];
}

template <typename T>
void launch_step_rhs(const Problem& P, const Dev<T>& D, const T* z, const T* y, int s, T* rhs, T cf,
                     hipStream_t st) {
    const int bs = 256;
    hipLaunchKernelGGL(step_rhs<T>, dim3((unsigned)((P.Nd + bs - 1) / bs)), dim3(bs), 0, st, z, y, D.gamma1,
                       D.gamma2, D.epad, s, P.M, P.Nd, cf, rhs);
    TSFDE_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Transposed operators (adjoint problem).  With w_s = gamma1^(s) .* lam^(s):
//   (A^T lam)^(m) = e_0 w_m + sum_{s=m+1}^{M-1} e_{s-m} w_s + [m = M-1] lam^(M)
//                   + c_t B (gamma2^(m) .* lam^(m))                          (m < M)
//   (A^T lam)^(M) = -eta sum_{s<M} q_s lam^(s) + c_f B (gamma2^(M-1) .* lam^(M))
// history_adj writes every term but the B products.  One thread per point; the outputs are taken
// kAdjTile time levels at a time (their sums in registers) while the inputs s >= m0 stream past.
// ---------------------------------------------------------------------------
constexpr int kAdjTile = 32;
static_assert(kAdjTile <= kEpad, "the tile overhang reads the leading zeros of epad");

template <typename T>
__global__ __launch_bounds__(256) void history_adj(const T* __restrict__ lam, T* __restrict__ z,
                                                   const T* __restrict__ g1, const T* __restrict__ epad,
                                                   const T* __restrict__ q, T eta, long long Nd, int M) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Nd) return;
    const T* e = epad + kEpad;  // e[k] = 0 for -kEpad <= k < 0
    T fr = T(0);
    for (int s = 0; s < M; ++s) fr += q[s] * lam[(long long)s * Nd + j];
    z[(long long)M * Nd + j] = -eta * fr;
    for (int m0 = 0; m0 < M; m0 += kAdjTile) {
        T acc[kAdjTile];
#pragma unroll
        for (int t = 0; t < kAdjTile; ++t) acc[t] = T(0);
        for (int s = m0; s < M; ++s) {
            const long long o = (long long)s * Nd + j;
            const T w = g1[o] * lam[o];
#pragma unroll
            for (int t = 0; t < kAdjTile; ++t) acc[t] += e[s - m0 - t] * w;  // zero for s < m0 + t
        }
#pragma unroll
        for (int t = 0; t < kAdjTile; ++t) {
            const int m = m0 + t;
            if (m < M) z[(long long)m * Nd + j] = acc[t] + (m == M - 1 ? lam[(long long)M * Nd + j] : T(0));
        }
    }
}

template <typename T>
void launch_history_adj(const Problem& P, const Dev<T>& D, const T* lam, T* z, hipStream_t s) {
    hipLaunchKernelGGL(history_adj<T>, dim3((unsigned)((P.Nd + 255) / 256)), dim3(256), 0, s, lam, z, D.gamma1,
                       D.epad, D.q, T(P.eta), P.Nd, P.M);
    TSFDE_HIP(hipGetLastError());
}

// only < 0: out^(s) = gamma2^(s) .* in^(s) for s < M and out^(M) = gamma2^(M-1) .* in^(M) (the inputs of
// the B products of A^T).  only >= 0: `in` is one slice and out^(only) = in (./ or .*) the gamma2 of
// that slice (gamma2^(M-1) for only = M).
template <typename T>
__global__ void scale_g2_k(const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ g2, long long Nd, int M,
                           int only, bool inverse) {
    const long long n = (only >= 0) ? Nd : (long long)(M + 1) * Nd;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long k = (only >= 0) ? (long long)only * Nd + i : i;  // index in the full vector
        const long long sl = k / Nd, j = k - sl * Nd;
        const T g = g2[(sl < M ? sl : M - 1) * Nd + j];
        const T v = in[(only >= 0) ? i : k];
        out[k] = inverse ? v / g : v * g;
    }
}

template <typename T>
void launch_scale_g2(const Problem& P, const Dev<T>& D, const T* in, T* out, int only, bool inverse, hipStream_t s) {
    const long long n = (only >= 0) ? P.Nd : P.ntot;
    hipLaunchKernelGGL(scale_g2_k<T>, dim3((unsigned)std::max(1LL, std::min<long long>((n + 255) / 256, 16384))),
                       dim3(256), 0, s, in, out, D.gamma2, P.Nd, P.M, only, inverse);
    TSFDE_HIP(hipGetLastError());
}

// right-hand side of backward-substitution step m (0-based) for P^T lam = g, in the variable u = gamma2 .* lam:
//   m < M : rhs = g^(m) - sum_{s=m+1}^{M-1} e_{s-m} gamma1^(s) .* lam^(s) - [m = M-1] lam^(M)
//   m = M : rhs = g^(M) / c_f
template <typename T>
__global__ void adj_step_rhs(const T* __restrict__ g, const T* __restrict__ lam, const T* __restrict__ g1,
                             const T* __restrict__ epad, int m, int M, long long Nd, T cf, T* __restrict__ rhs) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Nd) return;
    if (m == M) {
        rhs[j] = g[(long long)M * Nd + j] / cf;
        return;
    }
    const T* e = epad + kEpad;
    T h = T(0);
    for (int s = m + 1; s < M; ++s) {
        const long long o = (long long)s * Nd + j;
        h += e[s - m] * g1[o] * lam[o];
    }
    if (m == M - 1) h += lam[(long long)M * Nd + j];
    rhs[j] = g[(long long)m * Nd + j] - h;
}

// dL/dgamma2 from lam and v = (c_t B y^(s) for s < M, c_f B y^(M)):
//   G^(s) = -lam^(s) .* v^(s) (s < M), and G^(M-1) -= lam^(M) .* v^(M)
__global__ void gamma2_grad_k(const double* __restrict__ lam, const double* __restrict__ v, double* __restrict__ G,
                              long long Nd, int M) {
    const long long n = (long long)M * Nd;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        double g = -lam[i] * v[i];
        if (i >= (long long)(M - 1) * Nd) g -= lam[i + Nd] * v[i + Nd];
        G[i] = g;
    }
}
void launch_gamma2_grad(const Problem& P, const double* lam, const double* v, double* G, hipStream_t st) {
    const long long n = (long long)P.M * P.Nd;
    hipLaunchKernelGGL(gamma2_grad_k, dim3((unsigned)std::max(1LL, std::min<long long>((n + 255) / 256, 16384))),
                       dim3(256), 0, st, lam, v, G, P.Nd, P.M);
    TSFDE_HIP(hipGetLastError());
}

template <typename T>
void launch_adj_step_rhs(const Problem& P, const Dev<T>& D, const T* g, const T* lam, int m, T* rhs, hipStream_t st) {
    hipLaunchKernelGGL(adj_step_rhs<T>, dim3((unsigned)((P.Nd + 255) / 256)), dim3(256), 0, st, g, lam, D.gamma1,
                       D.epad, m, P.M, P.Nd, T(P.cf), rhs);
    TSFDE_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
template <typename T>
__global__ void dot_partials(const T* __restrict__ a, const T* __restrict__ b, long long n, T* __restrict__ partials) {
    __shared__ T red[4];
    T acc = T(0);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        acc += a[i] * b[i];
    T s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

static int blocks_for(long long n, int bs, int cap) {
    long long b = (n + bs - 1) / bs;
    return (int)std::max(1LL, std::min<long long>(b, cap));
}

template <typename T>
void launch_dot_partials(const T* a, const T* b, long long n, T* partials, int* nparts, hipStream_t s) {
    const int nb = blocks_for(n, 256, 1024);
    hipLaunchKernelGGL(dot_partials<T>, dim3(nb), dim3(256), 0, s, a, b, n, partials);
    TSFDE_HIP(hipGetLastError());
    *nparts = nb;
}

template <typename T>
__global__ void sum_partials_k(const T* __restrict__ partials, int n, double* __restrict__ out) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += (double)partials[i];
    double s = block_sum(acc, red);
    if (threadIdx.x == 0) *out = s;
}

void launch_sum_partials(const double* partials, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_partials_k<double>, dim3(1), dim3(256), 0, s, partials, n, out);
    TSFDE_HIP(hipGetLastError());
}
void launch_sum_partials(const float* partials, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_partials_k<float>, dim3(1), dim3(256), 0, s, partials, n, out);
    TSFDE_HIP(hipGetLastError());
}

// CG scalars, one thread.  scal: [0] rz  [1] pq  [2] alpha  [3] rr  [4] beta  [5] rz_new
__global__ void cg_scalars_k(double* scal, int mode) {
    if (threadIdx.x != 0) return;
    if (mode == 0) {  // alpha = rz / pq
        scal[2] = scal[1] != 0.0 ? scal[0] / scal[1] : 0.0;
    } else {          // beta = rz_new / rz ; rz = rz_new
        scal[4] = scal[0] != 0.0 ? scal[5] / scal[0] : 0.0;
        scal[0] = scal[5];
    }
}
void launch_cg_scalars(double* scal, int mode, hipStream_t s) {
    hipLaunchKernelGGL(cg_scalars_k, dim3(1), dim3(64), 0, s, scal, mode);
    TSFDE_HIP(hipGetLastError());
}

// x += alpha p ; r -= alpha q ; partials of (r, r)
template <typename T>
__global__ void cg_update_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
                             const double* __restrict__ scal, long long n, T* __restrict__ partials) {
    __shared__ T red[4];
    const T al = T(scal[2]);
    T acc = T(0);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        x[i] += al * p[i];
        const T rv = r[i] - al * q[i];
        r[i] = rv;
        acc += rv * rv;
    }
    T s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
template <typename T>
void launch_cg_update_xr(T* x, T* r, const T* p, const T* q, const double* scal, long long n, T* partials, int* nparts,
                         hipStream_t s) {
    const int nb = blocks_for(n, 256, 512);
    hipLaunchKernelGGL(cg_update_xr<T>, dim3(nb), dim3(256), 0, s, x, r, p, q, scal, n, partials);
    TSFDE_HIP(hipGetLastError());
    *nparts = nb;
}

// p = z + beta p
template <typename T>
__global__ void cg_update_p(T* __restrict__ p, const T* __restrict__ z, const double* __restrict__ scal, long long n) {
    const T be = T(scal[4]);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = z[i] + be * p[i];
}
template <typename T>
void launch_cg_update_p(T* p, const T* z, const double* scal, long long n, hipStream_t s) {
    const int nb = blocks_for(n, 256, 1024);
    hipLaunchKernelGGL(cg_update_p<T>, dim3(nb), dim3(256), 0, s, p, z, scal, n);
    TSFDE_HIP(hipGetLastError());
}

template <typename T>
__global__ void copy_k(const T* __restrict__ a, T* __restrict__ b, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = a[i];
}
template <typename T>
void launch_copy(const T* a, T* b, long long n, hipStream_t s) {
    hipLaunchKernelGGL(copy_k<T>, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, a, b, n);
    TSFDE_HIP(hipGetLastError());
}

template <typename A, typename B>
__global__ void convert_k(const A* __restrict__ a, B* __restrict__ b, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (B)a[i];
}
void launch_d2f(const double* a, float* b, long long n, hipStream_t s) {
    hipLaunchKernelGGL((convert_k<double, float>), dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, a, b, n);
    TSFDE_HIP(hipGetLastError());
}
void launch_f2d(const float* a, double* b, long long n, hipStream_t s) {
    hipLaunchKernelGGL((convert_k<float, double>), dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, a, b, n);
    TSFDE_HIP(hipGetLastError());
}

template <typename T>
__global__ void fill_k(T* p, long long n, T v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}
void launch_fill(double* p, long long n, double v, hipStream_t s) {
    hipLaunchKernelGGL(fill_k<double>, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
    TSFDE_HIP(hipGetLastError());
}
void launch_fill(float* p, long long n, float v, hipStream_t s) {
    hipLaunchKernelGGL(fill_k<float>, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
    TSFDE_HIP(hipGetLastError());
}
void launch_fill(unsigned long long* p, long long n, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(fill_k<unsigned long long>, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
    TSFDE_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Arnoldi helpers (FP64): classical Gram-Schmidt with one reorthogonalisation over the basis
// V[0..k) (k rows of n, row-major), in three passes over V:
//   multidot       h1 = V^T w
//   cgs_sub_dot    w -= V h1, then h2 = V^T w, from the same loads of V
//   cgs_sub_norm   w -= V h2, then ||w||^2
// Each pass splits n into gridDim.x contiguous chunks, one per block, and writes per-block partial
// sums partials[t * gridDim.x + block]; multidot_finish adds them in a fixed order.  Row indices past
// k - 1 are clamped to k - 1 (their coefficients are zero, their sums unused), so that a thread's
// loads of one element carry no branches and are all in flight together.
// ---------------------------------------------------------------------------
constexpr int kArnBlock = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    return v;
}

// h = V^T w: the block's 4 waves split the rows (RT per wave, the last wave's clamped), each wave
// sweeps the whole chunk and owns its rows' sums, so no block-wide reduction is needed.
template <int RT>
__global__ __launch_bounds__(kArnBlock) void multidot_k(const double* __restrict__ V, long long n, int k,
                                                        const double* __restrict__ w, double* __restrict__ partials) {
    const int lane = threadIdx.x & (kWave - 1);
    const int t0 = (threadIdx.x / kWave) * RT;
    if (t0 >= k) return;  // wave-uniform
    const long long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    const double* row[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) row[r] = V + (long long)min(t0 + r, k - 1) * n;
    double acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = 0.0;
    for (long long i = lo + lane; i < hi; i += kWave) {
        double v[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) v[r] = row[r][i];
        const double wv = w[i];
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r] += v[r] * wv;
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const double sum = wave_sum(acc[r]);
        if (lane == 0 && t0 + r < k) partials[(long long)(t0 + r) * gridDim.x + blockIdx.x] = sum;
    }
}

// Sums acc[t] (t < kk) over the block; thread t writes the total to out[t * ostride].
// red holds (kArnBlock / 64) * KB doubles.
template <int KB>
__device__ __forceinline__ void block_sum_multi(const double (&acc)[KB], int kk, double* red, double* out,
                                                long long ostride) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int t = 0; t < KB; ++t) {
        if (t < kk) {
            const double v = wave_sum(acc[t]);
            if (lane == 0) red[wid * KB + t] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < kk) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kArnBlock / kWave; ++q) s += red[q * KB + threadIdx.x];
        out[threadIdx.x * ostride] = s;
    }
    __syncthreads();
}

// Loads h[0..k) into hs[0..KB), zero past k
template <int KB>
__device__ __forceinline__ void load_coeffs(const double* h, int k, double* hs) {
    if ((int)threadIdx.x < KB) hs[threadIdx.x] = (int)threadIdx.x < k ? h[threadIdx.x] : 0.0;
    __syncthreads();
}

// w -= V h; then partials of V^T w (the reorthogonalisation's coefficients), k <= KB
template <int KB>
__global__ __launch_bounds__(kArnBlock) void cgs_sub_dot_k(const double* __restrict__ V, long long n, int k,
                                                           const double* __restrict__ h, double* __restrict__ w,
                                                           double* __restrict__ partials) {
    __shared__ double red[(kArnBlock / kWave) * KB];
    __shared__ double hs[KB];
    load_coeffs<KB>(h, k, hs);
    const long long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    double acc[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) acc[t] = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += kArnBlock) {
        double v[KB];
#pragma unroll
        for (int t = 0; t < KB; ++t) v[t] = V[(long long)min(t, k - 1) * n + i];
        double s = w[i];
#pragma unroll
        for (int t = 0; t < KB; ++t) s -= v[t] * hs[t];
        w[i] = s;
#pragma unroll
        for (int t = 0; t < KB; ++t) acc[t] += v[t] * s;
    }
    block_sum_multi<KB>(acc, k, red, partials + blockIdx.x, gridDim.x);
}

// w -= V h; then the partial sums of w . w, k <= KB
template <int KB>
__global__ __launch_bounds__(kArnBlock) void cgs_sub_norm_k(const double* __restrict__ V, long long n, int k,
                                                            const double* __restrict__ h, double* __restrict__ w,
                                                            double* __restrict__ partials) {
    __shared__ double red[kArnBlock / kWave];
    __shared__ double hs[KB];
    load_coeffs<KB>(h, k, hs);
    const long long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    double acc = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += kArnBlock) {
        double v[KB];
#pragma unroll
        for (int t = 0; t < KB; ++t) v[t] = V[(long long)min(t, k - 1) * n + i];
        // keep every load ahead of the dependent chain below
        __builtin_amdgcn_sched_barrier(0);
        double s = w[i];
#pragma unroll
        for (int t = 0; t < KB; ++t) s -= v[t] * hs[t];
        w[i] = s;
        acc += s * s;
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Launches KERNEL<X> for the smallest X = STEP, 2 STEP, ..., MAX with X >= need
template <int X, int STEP, int MAX, typename F>
static void launch_tier(int need, F&& f) {
    if constexpr (X >= MAX) {
        f(std::integral_constant<int, MAX>{});
    } else {
        if (need <= X) f(std::integral_constant<int, X>{});
        else launch_tier<X + STEP, STEP, MAX>(need, f);
    }
}

static void check_arnoldi(long long n, int k, int nblk) {
    if (k < 1 || k > kArnMaxK || nblk < 1 || n < 1)
        throw HipError{hipErrorInvalidValue, "Arnoldi pass: need 1 <= k <= kArnMaxK, n >= 1, nblk >= 1"};
}
static_assert(kArnMaxK == 4 * 16 && kArnMaxK % 8 == 0, "Arnoldi tiers cover kArnMaxK rows");

void launch_multidot(const double* V, long long n, int k, const double* w, double* partials, int nblk, hipStream_t s) {
    check_arnoldi(n, k, nblk);
    launch_tier<1, 1, 16>((k + 3) / 4, [&](auto rt) {
        hipLaunchKernelGGL(multidot_k<decltype(rt)::value>, dim3(nblk), dim3(kArnBlock), 0, s, V, n, k, w, partials);
    });
    TSFDE_HIP(hipGetLastError());
}
void launch_cgs_sub_dot(const double* V, long long n, int k, const double* h, double* w, double* partials, int nblk,
                        hipStream_t s) {
    check_arnoldi(n, k, nblk);
    launch_tier<8, 8, kArnMaxK>(k, [&](auto kb) {
        hipLaunchKernelGGL(cgs_sub_dot_k<decltype(kb)::value>, dim3(nblk), dim3(kArnBlock), 0, s, V, n, k, h, w,
                           partials);
    });
    TSFDE_HIP(hipGetLastError());
}
void launch_cgs_sub_norm(const double* V, long long n, int k, const double* h, double* w, double* partials, int nblk,
                         hipStream_t s) {
    check_arnoldi(n, k, nblk);
    launch_tier<8, 8, kArnMaxK>(k, [&](auto kb) {
        hipLaunchKernelGGL(cgs_sub_norm_k<decltype(kb)::value>, dim3(nblk), dim3(kArnBlock), 0, s, V, n, k, h, w,
                           partials);
    });
    TSFDE_HIP(hipGetLastError());
}

// h[t] = sum_b partials[t * nblk + b], one block per t
__global__ void multidot_finish_k(const double* __restrict__ partials, int nblk, double* __restrict__ h) {
    __shared__ double red[4];
    const double* p = partials + (long long)blockIdx.x * nblk;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += p[b];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) h[blockIdx.x] = s;
}
void launch_multidot_finish(const double* partials, int nblk, int k, double* h, hipStream_t s) {
    hipLaunchKernelGGL(multidot_finish_k, dim3(k), dim3(256), 0, s, partials, nblk, h);
    TSFDE_HIP(hipGetLastError());
}

// x += Z[0..k) y
__global__ void gemv_add_k(const double* __restrict__ Z, long long n, int k, const double* __restrict__ y,
                           double* __restrict__ x) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        double acc = x[i];
        for (int t = 0; t < k; ++t) acc += Z[(long long)t * n + i] * y[t];
        x[i] = acc;
    }
}
void launch_gemv_add(const double* Z, long long n, int k, const double* y, double* x, hipStream_t s) {
    hipLaunchKernelGGL(gemv_add_k, dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, Z, n, k, y, x);
    TSFDE_HIP(hipGetLastError());
}

// v *= 1/den  (den a device scalar holding a norm)
__global__ void scale_k(double* __restrict__ v, long long n, const double* __restrict__ den) {
    const double inv = 1.0 / (*den);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        v[i] *= inv;
}
void launch_scale(double* v, long long n, const double* num, const double* den, hipStream_t s) {
    (void)num;
    hipLaunchKernelGGL(scale_k, dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, v, n, den);
    TSFDE_HIP(hipGetLastError());
}

// The transposed sweep's inputs in reversed step order: zrev_k = g^(M-1-k) (k = 0: minus lam^(M), the
// coupling of the last block row), dgrev_k = dg_{M-1-k}, k < M
__global__ void adj_reverse_k(const double* __restrict__ g, const double* __restrict__ lam,
                              const double* __restrict__ dg, double* __restrict__ zrev, double* __restrict__ dgrev,
                              long long Nd, int M) {
    const long long n = (long long)M * Nd;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long k = i / Nd, j = i - k * Nd;
        const long long src = (long long)(M - 1 - k) * Nd + j;
        double zv = g[src];
        if (k == 0) zv -= lam[(long long)M * Nd + j];
        zrev[i] = zv;
        dgrev[i] = dg[src];
    }
}
void launch_adj_reverse(const Problem& P, const double* g, const double* lam, double* zrev, double* dgrev,
                        hipStream_t s) {
    const long long n = (long long)P.M * P.Nd;
    hipLaunchKernelGGL(adj_reverse_k, dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, g, lam, P.f64.dg, zrev, dgrev,
                       P.Nd, P.M);
    TSFDE_HIP(hipGetLastError());
}

// lam^(m) = urev_{M-1-m} ./ gamma2^(m) for m < M, in place over lam's first M slices (urev): the thread
// of the pair (k, M-1-k) reads both before it writes either
__global__ void adj_unreverse_k(double* __restrict__ lam, const double* __restrict__ g2, long long Nd, int M) {
    const long long half = (long long)((M + 1) / 2) * Nd;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < half; i += (long long)gridDim.x * blockDim.x) {
        const long long k = i / Nd, j = i - k * Nd;
        const long long a = k * Nd + j, b = (long long)(M - 1 - k) * Nd + j;
        const double ua = lam[a], ub = lam[b];
        lam[a] = ub / g2[a];  // slice k from urev_{M-1-k}
        lam[b] = ua / g2[b];  // slice M-1-k from urev_k (the same point when k = M-1-k)
    }
}
void launch_adj_unreverse(const Problem& P, double* lam, hipStream_t s) {
    const long long n = (long long)((P.M + 1) / 2) * P.Nd;
    hipLaunchKernelGGL(adj_unreverse_k, dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, lam, P.f64.gamma2, P.Nd,
                       P.M);
    TSFDE_HIP(hipGetLastError());
}

__global__ void scale_rsqrt_k(double* __restrict__ v, long long n, const double* __restrict__ sq) {
    const double q = *sq;
    const double inv = (q > 0.0 && q <= 1.79e308) ? 1.0 / sqrt(q) : 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        v[i] *= inv;
}
void launch_scale_rsqrt(double* v, long long n, const double* sq, hipStream_t s) {
    hipLaunchKernelGGL(scale_rsqrt_k, dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, v, n, sq);
    TSFDE_HIP(hipGetLastError());
}

__global__ void axpby_k(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = a * x[i] + b * y[i];
}
// The last block column of A that P drops (§5.1): P v = A v + eta (q (x) I) v^(M) in the block rows
// s < M; transposed, P^T u = A^T u + eta sum_{s < M} q_s u^(s) in the last block row.
__global__ void coupling_k(double* __restrict__ out, const double* __restrict__ v, const double* __restrict__ q,
                           double eta, long long Nd, int M, int transpose) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Nd) return;
    if (transpose) {
        double acc = 0.0;
        for (int s = 0; s < M; ++s) acc += q[s] * v[(long long)s * Nd + j];
        out[(long long)M * Nd + j] += eta * acc;
    } else {
        const double f = eta * v[(long long)M * Nd + j];
        for (int s = 0; s < M; ++s) out[(long long)s * Nd + j] += q[s] * f;
    }
}

void launch_coupling(const Problem& P, const double* v, double* out, bool transpose, hipStream_t s) {
    hipLaunchKernelGGL(coupling_k, dim3((unsigned)((P.Nd + 255) / 256)), dim3(256), 0, s, out, v, P.f64.q, P.eta,
                       P.Nd, P.M, transpose ? 1 : 0);
    TSFDE_HIP(hipGetLastError());
}

// x_i = a uniform value in [-1, 1) from a 64-bit hash of (seed, i) (splitmix64): a start vector with
// components along every singular direction
__global__ void hash_fill_k(double* __restrict__ x, long long n, unsigned long long seed) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

void launch_hash_fill(double* x, long long n, unsigned long long seed, hipStream_t s) {
    hipLaunchKernelGGL(hash_fill_k, dim3(blocks_for(n, 256, 1 << 30)), dim3(256), 0, s, x, n, seed);
    TSFDE_HIP(hipGetLastError());
}

void launch_axpby(double a, const double* x, double b, const double* y, double* out, long long n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_k, dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, a, x, b, y, out, n);
    TSFDE_HIP(hipGetLastError());
}

// z = [b_{s-1} gamma1^(s) rho ; mu]   (eq. lin-syst right-hand side)
__global__ void build_z_k(const double* __restrict__ g1, const double* __restrict__ bw, const double* __restrict__ rho,
                          const double* __restrict__ mu, long long Nd, int M, double* __restrict__ z) {
    const long long n = (long long)(M + 1) * Nd;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long s = i / Nd, j = i - s * Nd;
        z[i] = (s < M) ? bw[s] * g1[i] * rho[j] : mu[j];
    }
}
// z-hat = b_{s-1} gamma1^(s) rho + eta q^(s) f, s = 1..M, plus a zero last block
__global__ void build_zhat_k(const double* __restrict__ g1, const double* __restrict__ bw,
                             const double* __restrict__ rho, const double* __restrict__ q, const double* __restrict__ f,
                             double eta, long long Nd, int M, double* __restrict__ z) {
    const long long n = (long long)(M + 1) * Nd;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long s = i / Nd, j = i - s * Nd;
        z[i] = (s < M) ? bw[s] * g1[i] * rho[j] + eta * q[s] * f[j] : 0.0;
    }
}

void launch_build_z(const Problem& P, double* z, hipStream_t s, const double* mu) {
    const long long n = P.ntot;
    hipLaunchKernelGGL(build_z_k, dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, P.f64.gamma1, P.d_bw, P.d_rho,
                       mu ? mu : P.d_mu, P.Nd, P.M, z);
    TSFDE_HIP(hipGetLastError());
}
void launch_build_zhat(const Problem& P, const double* f, double* zhat, hipStream_t s) {
    const long long n = P.ntot;
    hipLaunchKernelGGL(build_zhat_k, dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, P.f64.gamma1, P.d_bw, P.d_rho,
                       P.f64.q, f, P.eta, P.Nd, P.M, zhat);
    TSFDE_HIP(hipGetLastError());
}

// out = a - b, partials of (out, out)
template <typename T>
__global__ void sub_partials_k(const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ out, long long n,
                               T* __restrict__ partials) {
    __shared__ T red[4];
    T acc = T(0);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const T v = a[i] - b[i];
        out[i] = v;
        acc += v * v;
    }
    T s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
template <typename T>
void launch_sub_partials(const T* a, const T* b, T* out, long long n, T* partials, int* nparts, hipStream_t s) {
    const int nb = blocks_for(n, 256, 512);
    hipLaunchKernelGGL(sub_partials_k<T>, dim3(nb), dim3(256), 0, s, a, b, out, n, partials);
    TSFDE_HIP(hipGetLastError());
    *nparts = nb;
}

// z = r / (dg + c a0), partials of (r, z)   (diagonal preconditioner when the sine transform is unavailable)
template <typename T>
__global__ void jacobi_prec_k(const T* __restrict__ r, T* __restrict__ z, const T* __restrict__ dg, T c, T a0,
                              long long n, T* __restrict__ partials) {
    __shared__ T red[4];
    T acc = T(0);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const T v = r[i] / ((dg ? dg[i] : T(0)) + c * a0);
        z[i] = v;
        acc += r[i] * v;
    }
    T s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
template <typename T>
void launch_jacobi_prec(const T* r, T* z, const T* dg, T c, T a0, long long n, T* partials, int* nparts,
                        hipStream_t s) {
    const int nb = blocks_for(n, 256, 512);
    hipLaunchKernelGGL(jacobi_prec_k<T>, dim3(nb), dim3(256), 0, s, r, z, dg, c, a0, n, partials);
    TSFDE_HIP(hipGetLastError());
    *nparts = nb;
}

}  // namespace tsfde

// explicit instantiations
namespace tsfde {
template void launch_history_matvec<double>(const Problem&, const Dev<double>&, const double*, double*, hipStream_t);
template void launch_history_adj<double>(const Problem&, const Dev<double>&, const double*, double*, hipStream_t);
template void launch_scale_g2<double>(const Problem&, const Dev<double>&, const double*, double*, int, bool,
                                      hipStream_t);
template void launch_adj_step_rhs<double>(const Problem&, const Dev<double>&, const double*, const double*, int,
                                          double*, hipStream_t);
template void launch_history_matvec<float>(const Problem&, const Dev<float>&, const float*, float*, hipStream_t);
template void launch_step_rhs<double>(const Problem&, const Dev<double>&, const double*, const double*, int, double*,
                                      double, hipStream_t);
template void launch_step_rhs<float>(const Problem&, const Dev<float>&, const float*, const float*, int, float*, float,
                                     hipStream_t);
template void launch_dot_partials<double>(const double*, const double*, long long, double*, int*, hipStream_t);
template void launch_dot_partials<float>(const float*, const float*, long long, float*, int*, hipStream_t);
template void launch_cg_update_xr<double>(double*, double*, const double*, const double*, const double*, long long,
                                          double*, int*, hipStream_t);
template void launch_cg_update_xr<float>(float*, float*, const float*, const float*, const double*, long long, float*,
                                         int*, hipStream_t);
template void launch_cg_update_p<double>(double*, const double*, const double*, long long, hipStream_t);
template void launch_cg_update_p<float>(float*, const float*, const double*, long long, hipStream_t);
template void launch_copy<double>(const double*, double*, long long, hipStream_t);
template void launch_copy<float>(const float*, float*, long long, hipStream_t);
template void launch_sub_partials<double>(const double*, const double*, double*, long long, double*, int*, hipStream_t);
template void launch_sub_partials<float>(const float*, const float*, float*, long long, float*, int*, hipStream_t);
template void launch_jacobi_prec<double>(const double*, double*, const double*, double, double, long long, double*,
                                         int*, hipStream_t);
template void launch_jacobi_prec<float>(const float*, float*, const float*, float, float, long long, float*, int*,
                                        hipStream_t);
}  // namespace tsfde
