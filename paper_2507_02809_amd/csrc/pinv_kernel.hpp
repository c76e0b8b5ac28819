// P^{-1} z with persistent kernels (§5.1 'Implementation': forward substitution over
// the time steps; each diagonal block solved by preconditioned CG on its symmetrised form).
//
// The forward substitution is a chain of M+1 dependent solves on one spatial slice each, and every
// CG iteration is a handful of small transforms and two reductions.  Launching those as separate
// kernels costs microseconds per launch plus a host round trip per convergence test, so here a
// persistent grid of G workgroups runs a segment of up to kHB consecutive steps, separating
// phases with a device-wide barrier and taking every convergence decision on the device: all
// workgroups reduce the same partial sums in the same order and take the same branch.
//
// Between segments an ordinary full-GPU kernel sums the "far" part of the time history and folds
// it into the right-hand side of each step s = sa + i of the segment,
//   w_s = (z_s - gamma1_s sum_{m < sa} e_{s-m} y_m) / gamma2_s,   i < kHB,
// a bandwidth-bound block Toeplitz product over all earlier slices; inside a segment each step
// adds only the near terms m in [sa, s): rhs_s = w_s - (gamma1_s/gamma2_s) sum_{sa <= m < s} e_{s-m} y_m.
//
// Per step s (0-based; s = M is the last block row), 2D with the sine-transform preconditioner:
//   [E+A]  per row pair: finish step s-1 (y_{s-1} = x, B y_{s-1} recovered from its residual),
//          history, rhs = (z_s - gamma1 hist)/gamma2, warm start x0 = 2 y_{s-1} - y_{s-2},
//          r0 = rhs - A_s x0, (r0, r0), (rhs, rhs); sine transform of the r0 rows -> t1
//   [B]    second sine transform, spectral scaling, third transform -> t2; (r, z)
//   loop { [DF]  last transform of z = M^{-1} r, p = z + beta p, (p, dg p), row FFT of p
//          [C]   column FFT, symbol, inverse column FFT; (p, B p)
//          [IUA] inverse row FFT -> B p; x += alpha p, r -= alpha q, (r, r); sine transform of r
//          check; [B] }
// i.e. four device-wide barriers per CG iteration.  The 1D problem and the 2D problem with the
// diagonal preconditioner run a simpler chain (E, then rows/columns/rows of q = A_s p).
// Every phase issues its global loads before its stores, so that a thread's independent memory
// accesses overlap instead of waiting one cache miss at a time.
//
// This header holds the device code and the launch template; the kernels are instantiated in
// pinv_persistent.hip (transform length a run-time value) and pinv_fixed.hip (the 2D
// sine-transform path with the length a compile-time constant, which lets the compiler fold the
// FFT's pass structure and LDS addressing).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "fft.hpp"
#include "grid_sync.hpp"
#include "internal.hpp"
#include "residency.hpp"

namespace tsfde {

static_assert(kHB <= 64, "the weight table e carries 64 trailing zeros for the history tiles");
constexpr int kNPart = 6;  // reduction slots per workgroup
// near-history terms of a step of the segment kernel: y_m with sa <= m < s - 1 and s - sa <= kHB - 1
constexpr int kNear = kHB - 2;
// (r,r) (rhs,rhs) (r,z) (p,q) (p,dg p) (p,B p)
enum : int { SL_RR = 0, SL_BB = 1, SL_RZ = 2, SL_PQ = 3, SL_PD = 4, SL_PB = 5 };

template <typename T>
struct PinvArgs {
    int d, N, M, L, H;
    int ns;  // row stride of the transposed 2D intermediates spec, t1, t2 (N rounded up to 16)
    long long Nd;
    int use_tau;  // 1: tau (sine transform) preconditioner, 0: diagonal
    int Nt;       // size of the sine transform: N, or the padded size with L = 2 (Nt + 1)
    int nt;       // 2D: row stride of the sine-transform intermediates t1 [Nt][nt], t2 [N][nt]
    int extrap;   // block CG initial guess: 0 previous level, 1 linear, 2 quadratic, 3 half-linear extrapolation
    int adj;      // 1: the transposed sweep (history weights per earlier step: rhs = w - sum e dg_m y_m)
    const T* z;
    T* y;
    const T* g1;
    const T* g2;
    const T* dg;
    const T* epad;
    const T* sym;
    const T* tau;
    const cplx<T>* tw;
    const double* sigma;  // [M]
    T ct, cf, a0;
    double tol2;
    int maxit;
    // work (Nd each unless noted)
    T *x, *r, *zz, *p, *q, *t1, *t2, *rhs, *bxb, *bxb2;  // bxb, bxb2: B y_{s-2}, B y_{s-3} (warm start)
    T* hacc;           // [kHB][Nd]: w_s of the segment's steps (far history folded into the rhs)
    cplx<T>* spec;     // [H][ns]
    double* part;      // [kRing][kMaxGrid][kNPart] reduction slots (phase_sync)
    unsigned* bar;     // [1] abort word (see grid_barrier_n)
    unsigned long long bar_ticks;  // longest barrier wait, in wall-clock periods
    long long* iters;  // accumulated CG iterations
    int vb, vg;        // this workgroup's index in the problem's grid and that grid's size
    int ring;          // 1: the segment's earlier solutions of the thread's own points kept in LDS (2D tau
                       // path with one round over the row pairs; near-history terms read from there)
};

// (A problem's workgroups are numbered vb = 0 .. vg - 1 within its grid: the whole launch, or its share
// of a launch that runs several problems side by side.)

// ---------------------------------------------------------------------------
// Phase synchronisation of the segment kernel: the device-wide barrier and the reduction of the
// phase's partial sums in one exchange.
//
// part holds kRing rings of [kMaxGrid][kNPart] slots; phase ph uses ring ph % kRing.  A slot is
// empty (the bit pattern kEmpty) until its workgroup publishes the phase's value there, so a
// workgroup has arrived at the barrier of phase ph once its slots of that phase are filled, and the
// waiting workgroups read the values they reduce in the same loads that tell them so (no arrival
// counter, no second round trip for the partial sums).  When it publishes phase ph, a workgroup
// first empties its slots of ring ph + 1; a release fence orders that, and every store of the phase,
// before the published values.  Ring ph + 1 was last read in phase ph - 3 (by a gather of that phase
// or of the next one), and every workgroup has finished those reads before publishing phase ph - 1,
// which the publishing workgroup has seen.  The launch starts at phase 0 with ring 0 emptied by the
// host.  kEmpty is a NaN payload that arithmetic does not produce (an operation on finite values
// that yields NaN gives the default NaN); a slot holding it by accident would end in the bounded
// wait's time-out, not in a wrong sum.
//
// The wait is bounded as in grid_barrier_n (bar[1] is the abort word).  The additions are in a fixed
// order (a shuffle tree per wave, the waves in order; then lane b of one wave adds workgroups b,
// b + 64, ... and a shuffle tree adds the lanes), the same in every workgroup, so every workgroup
// takes the same branches and results do not change with timing.
// ---------------------------------------------------------------------------
constexpr int kRing = 4;
constexpr int kMaxGrid = 256;  // workgroups of one problem's grid at most (the ring stride)
constexpr unsigned long long kEmpty = 0x7FF4DEAD7FF4DEADull;

__device__ __forceinline__ unsigned long long* ring_slot(double* part, unsigned ph, int b, int k) {
    return reinterpret_cast<unsigned long long*>(part + ((size_t)(ph % kRing) * kMaxGrid + b) * kNPart + k);
}

// Publish the K values (slots slot[k]) of this workgroup for phase ph, wait until all G workgroups
// have published theirs, and (GATH) leave the totals in tot[] for all threads; PREV >= 0 also
// gathers that slot from phase ph - 1 (published there without a gather).  VALS = false: a barrier
// only (the value published marks the arrival; tot is left alone).  Advances ph.
template <int K, bool GATH, int PREV, typename T, bool VALS = true>
__device__ __forceinline__ void phase_sync(double* part, unsigned* bar, unsigned long long ticks, const int (&slot)[K],
                                           const T (&val)[K], double* red, double* tot, unsigned& ph, int vb, int G) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    {
        const int nact = min(kWave, (int)blockDim.x - wid * kWave);
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = (double)val[k];
        for (int off = kWave / 2; off > 0; off >>= 1) {
            double o[K];
#pragma unroll
            for (int k = 0; k < K; ++k) o[k] = __shfl_down(v[k], off, kWave);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (lane + off < nact) v[k] += o[k];
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) red[wid * K + k] = v[k];
        }
    }
    __syncthreads();  // red complete; every thread's stores of this phase issued before the release below
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + kWave - 1) / kWave;
        double r[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            r[k] = 0.0;
            for (int w = 0; w < nw; ++w) r[k] += red[w * K + k];
        }
        if (G <= 1) {
            // the only workgroup: its sums are the totals (a slot published without a gather is
            // kept in tot for the next phase's)
            if constexpr (VALS) {
#pragma unroll
                for (int k = 0; k < K; ++k) tot[slot[k]] = r[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < kNPart; ++k)
                __hip_atomic_store(ring_slot(part, ph + 1, vb, k), kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#pragma unroll
            for (int k = 0; k < K; ++k)
                __hip_atomic_store(ring_slot(part, ph, vb, slot[k]), (unsigned long long)__double_as_longlong(r[k]),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (G > 1 && wid == 0) {
        // lane l waits for workgroups l, l + 64, ...; the loads of a poll are in flight together
        constexpr int NB = kMaxGrid / kWave;
        unsigned long long got[NB][K], prv[NB];
        const unsigned long long t0 = (unsigned long long)wall_clock64();
        while (true) {
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = lane + i * kWave;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    got[i][k] = (b < G) ? __hip_atomic_load(ring_slot(part, ph, b, slot[k]), __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)
                                        : 0ull;
                if constexpr (PREV >= 0)
                    prv[i] = (b < G) ? __hip_atomic_load(ring_slot(part, ph - 1, b, PREV), __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)
                                     : 0ull;
            }
            const unsigned ab = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bool ready = true;
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int k = 0; k < K; ++k) ready = ready && got[i][k] != kEmpty;
            if (__all(ready)) break;
            if (ab != 0u) break;  // an earlier wait timed out: finish without waiting
            if ((unsigned long long)wall_clock64() - t0 > ticks) {
                if (lane == 0) __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if constexpr (GATH) {
            constexpr int KG = K + (PREV >= 0 ? 1 : 0);
            double v[KG];
#pragma unroll
            for (int k = 0; k < KG; ++k) v[k] = 0.0;
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                if (lane + i * kWave < G) {
#pragma unroll
                    for (int k = 0; k < K; ++k) v[k] += __longlong_as_double((long long)got[i][k]);
                    if constexpr (PREV >= 0) v[K] += __longlong_as_double((long long)prv[i]);
                }
            }
            for (int off = kWave / 2; off > 0; off >>= 1) {
                double o[KG];
#pragma unroll
                for (int k = 0; k < KG; ++k) o[k] = __shfl_down(v[k], off, kWave);
#pragma unroll
                for (int k = 0; k < KG; ++k)
                    if (lane + off < min(kWave, (int)blockDim.x)) v[k] += o[k];
            }
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < K; ++k) tot[slot[k]] = v[k];
                if constexpr (PREV >= 0) tot[PREV] = v[K];
            }
        }
    }
    __syncthreads();
    ++ph;
}

// a device-wide barrier of the segment kernel (phase_sync with no sums)
__device__ __forceinline__ void phase_barrier(double* part, unsigned* bar, unsigned long long ticks, double* red,
                                              double* tot, unsigned& ph, int vb, int G) {
    const int sl[1] = {0};
    const double vv[1] = {0.0};
    phase_sync<1, false, -1, double, false>(part, bar, ticks, sl, vv, red, tot, ph, vb, G);
}

// ---------------------------------------------------------------------------
// far history folded into the right-hand side: for i < cnt (<= kHB), s = sa + i < M,
//   w[i][j] = (z_s[j] - gamma1_s[j] sum_{m < sa} e_{s-m} y_m[j]) / gamma2_s[j],
// or, for the transposed sweep (g1 = g2 = null, dgcol = the per-step weights of the earlier steps),
//   w[i][j] = z_s[j] - sum_{m < sa} e_{s-m} dgcol_m[j] y_m[j].
// One workgroup = 64 points x 4 waves; wave w sums the steps m = w, w+4, ...
template <typename T>
__global__ __launch_bounds__(256) void far_history(const T* __restrict__ y, T* __restrict__ w_out,
                                                   const T* __restrict__ epad, const T* __restrict__ z,
                                                   const T* __restrict__ g1, const T* __restrict__ g2, int sa,
                                                   int cnt, long long Nd, const T* __restrict__ dgcol) {
    __shared__ T part[4][kHB][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const long long j = (long long)blockIdx.x * 64 + lane;
    const T* e = epad + kEpad;
    T acc[kHB];
#pragma unroll
    for (int i = 0; i < kHB; ++i) acc[i] = T(0);
    if (j < Nd) {
#pragma unroll 4
        for (int m = w; m < sa; m += 4) {
            T ym = y[(long long)m * Nd + j];
            if (dgcol) ym *= dgcol[(long long)m * Nd + j];
#pragma unroll
            for (int i = 0; i < kHB; ++i) acc[i] += e[sa + i - m] * ym;
        }
    }
#pragma unroll
    for (int i = 0; i < kHB; ++i) part[w][i][lane] = acc[i];
    __syncthreads();
    if (j < Nd) {
        // wave w finishes the steps i = w, w + 4, ...
        for (int i = w; i < cnt; i += 4) {
            const long long o = (long long)(sa + i) * Nd + j;
            const T h = (part[0][i][lane] + part[1][i][lane]) + (part[2][i][lane] + part[3][i][lane]);
            w_out[(long long)i * Nd + j] = g1 ? (z[o] - g1[o] * h) / g2[o] : z[o] - h;
        }
    }
}

// ---------------------------------------------------------------------------
// group-level transforms (a group = nthr threads sharing one LDS sequence of length L)
// ---------------------------------------------------------------------------

// 2D: rows (i0, i1) of p -> half spectra spec[k][i] (k < L/2+1), after p = zz + beta p
template <typename T, int VPT>
__device__ __forceinline__ void g_rows_fwd(const PinvArgs<T>& a, cplx<T>* c, const cplx<T>* tw, int pair, bool valid, T beta, int tid,
                           int nthr) {
    const int N = a.N, L = a.L;
    const int i0 = 2 * pair, i1 = i0 + 1;
    const bool two = i1 < N;
    T z0[VPT], z1[VPT], p0[VPT], p1[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int j = tid + u * nthr;
        z0[u] = z1[u] = p0[u] = p1[u] = T(0);
        if (valid && j < N) {
            const long long o0 = (long long)i0 * N + j;
            z0[u] = a.zz[o0];
            if (beta != T(0)) p0[u] = a.p[o0];
            if (two) {
                z1[u] = a.zz[o0 + N];
                if (beta != T(0)) p1[u] = a.p[o0 + N];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int j = tid + u * nthr;
        const T v0 = z0[u] + beta * p0[u], v1 = z1[u] + beta * p1[u];
        if (valid && j < N) {
            const long long o0 = (long long)i0 * N + j;
            a.p[o0] = v0;
            if (two) a.p[o0 + N] = v1;
        }
        c[lx(j)] = {v0, v1};
    }
    __syncthreads();
    fft_lds<T, VPT, false, true>(c, L, tw, tid, nthr);
    if (valid) {
        const int H = a.H;
        for (int k = tid; k < H; k += nthr) {
            const cplx<T> C = c[lx(k)];
            const cplx<T> Cm = c[lx((L - k) & (L - 1))];
            a.spec[(long long)k * a.ns + i0] = {T(0.5) * (C.x + Cm.x), T(0.5) * (C.y - Cm.y)};
            if (two) a.spec[(long long)k * a.ns + i1] = {T(0.5) * (C.y + Cm.y), T(0.5) * (Cm.x - C.x)};
        }
    }
    __syncthreads();
}

// 2D: spectral row k2: FFT over i, times the circulant symbol, inverse FFT over k1
template <typename T, int VPT>
__device__ __forceinline__ void g_cols(const PinvArgs<T>& a, cplx<T>* c, const cplx<T>* tw, int k2, bool valid, int tid, int nthr) {
    const int N = a.N, L = a.L;
    cplx<T>* row = a.spec + (long long)k2 * a.ns;
    const T* sy = a.sym + (long long)k2 * L;
    T sv[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int i = tid + u * nthr;
        c[lx(i)] = (valid && i < N) ? row[i] : cplx<T>{T(0), T(0)};
        sv[u] = valid ? sy[i] : T(0);
    }
    __syncthreads();
    fft_lds<T, VPT, false, true>(c, L, tw, tid, nthr);
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int k1 = tid + u * nthr;
        c[lx(k1)] = {c[lx(k1)].x * sv[u], c[lx(k1)].y * sv[u]};
    }
    __syncthreads();
    fft_lds<T, VPT, true, true>(c, L, tw, tid, nthr);
    if (valid) {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int i = tid + u * nthr;
            if (i < N) row[i] = c[lx(i)];
        }
    }
    __syncthreads();
}

// 2D: rows (i0, i1): inverse transform of the half spectra, q = dg p + c u, accumulate (p, q)
template <typename T, int VPT>
__device__ __forceinline__ void g_rows_inv(const PinvArgs<T>& a, cplx<T>* c, const cplx<T>* tw, int pair, bool valid, const T* dg,
                           T cc, int tid, int nthr, T& pq) {
    const int N = a.N, L = a.L, H = a.H;
    const int i0 = 2 * pair, i1 = i0 + 1;
    const bool two = i1 < N;
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int k = tid + u * nthr;
        cplx<T> v = {T(0), T(0)};
        if (valid) {
            const int kk = (k < H) ? k : L - k;
            const cplx<T> Y0 = a.spec[(long long)kk * a.ns + i0];
            const cplx<T> Y1 = two ? a.spec[(long long)kk * a.ns + i1] : cplx<T>{T(0), T(0)};
            v = (k < H) ? cplx<T>{Y0.x - Y1.y, Y0.y + Y1.x} : cplx<T>{Y0.x + Y1.y, Y1.x - Y0.y};
        }
        c[lx(k)] = v;
    }
    // loads of p and dg for the epilogue, in flight while the transform runs
    T p0[VPT], p1[VPT], d0[VPT], d1[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int j = tid + u * nthr;
        p0[u] = p1[u] = d0[u] = d1[u] = T(0);
        if (valid && j < N) {
            const long long o0 = (long long)i0 * N + j;
            p0[u] = a.p[o0];
            if (dg) d0[u] = dg[o0];
            if (two) {
                p1[u] = a.p[o0 + N];
                if (dg) d1[u] = dg[o0 + N];
            }
        }
    }
    __syncthreads();
    fft_lds<T, VPT, true, true>(c, L, tw, tid, nthr);
    if (valid) {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int j = tid + u * nthr;
            if (j < N) {
                const cplx<T> uu = c[lx(j)];
                const long long o0 = (long long)i0 * N + j;
                const T q0 = d0[u] * p0[u] + cc * uu.x;
                a.q[o0] = q0;
                pq += p0[u] * q0;
                if (two) {
                    const T q1 = d1[u] * p1[u] + cc * uu.y;
                    a.q[o0 + N] = q1;
                    pq += p1[u] * q1;
                }
            }
        }
    }
    __syncthreads();
}

// Sine transform (DST-I of size L/2 - 1 via the odd extension of length L) of rows (i0, i1) of `in`
// (N entries each, zero-padded when L/2 - 1 > N), with the two rows packed as real + i*imag;
// afterwards c[lx(k+1)] = -2i DST(row i0)_k + 2 DST(row i1)_k.
// With upd, first x += alpha p and in -= alpha q on those rows (accumulating (in, in)).
// d = 1: a single row.
template <typename T, int VPT>
__device__ __forceinline__ void g_dst_load(const PinvArgs<T>& a, cplx<T>* c, const cplx<T>* tw, T* in, int ld, int i0, bool valid,
                           int tid, int nthr, bool upd, T alpha, T& rr) {
    const int N = a.N, L = a.L;
    const bool two = (a.d == 2) && (i0 + 1 < N);
    constexpr int VH = VPT / 2;  // the odd extension's first half: m < L/2 = VH * nthr, and N < L/2
    T v0[VH], v1[VH];
    if (upd) {
        T q0[VH], q1[VH], x0[VH], x1[VH], pp0[VH], pp1[VH];
#pragma unroll
        for (int u = 0; u < VH; ++u) {
            const int m = tid + u * nthr;
            v0[u] = v1[u] = q0[u] = q1[u] = x0[u] = x1[u] = pp0[u] = pp1[u] = T(0);
            if (valid && m < N) {
                const long long o0 = (long long)i0 * ld + m;
                v0[u] = in[o0];
                q0[u] = a.q[o0];
                x0[u] = a.x[o0];
                pp0[u] = a.p[o0];
                if (two) {
                    v1[u] = in[o0 + ld];
                    q1[u] = a.q[o0 + ld];
                    x1[u] = a.x[o0 + ld];
                    pp1[u] = a.p[o0 + ld];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < VH; ++u) {
            const int m = tid + u * nthr;
            v0[u] -= alpha * q0[u];
            v1[u] -= alpha * q1[u];
            rr += v0[u] * v0[u] + v1[u] * v1[u];
            if (valid && m < N) {
                const long long o0 = (long long)i0 * ld + m;
                in[o0] = v0[u];
                a.x[o0] = x0[u] + alpha * pp0[u];
                if (two) {
                    in[o0 + ld] = v1[u];
                    a.x[o0 + ld] = x1[u] + alpha * pp1[u];
                }
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < VH; ++u) {
            const int m = tid + u * nthr;
            v0[u] = v1[u] = T(0);
            if (valid && m < N) {
                const long long o0 = (long long)i0 * ld + m;
                v0[u] = in[o0];
                if (two) v1[u] = in[o0 + ld];
            }
        }
    }
    // odd extension of length L: position m + 1 holds x_m and position L - 1 - m holds -x_m for
    // m < L/2 (zero past the data, m >= N: the padded entries and position L/2), position 0 is zero
#pragma unroll
    for (int u = 0; u < VH; ++u) {
        const int m = tid + u * nthr;
        c[lx(m + 1)] = {v0[u], v1[u]};
        c[lx(L - m - 1)] = {-v0[u], -v1[u]};
    }
    if (tid == 0) c[lx(0)] = {T(0), T(0)};
    __syncthreads();
    fft_lds<T, VPT, false, true>(c, L, tw, tid, nthr);
}

// Sine transform (size L/2 - 1) of rows (i0, i0 + 1) of `in` (n entries each, zero-padded up to
// L/2 - 1; row stride ld; the second row exists when i0 + 1 < nrow), packed as real + i*imag: the
// odd extension of length L is loaded from global memory straight into the FFT's register layout
// (thread tid: positions tid + u nthr), so only the transform's own exchanges use LDS.
// Afterwards c[lx(k+1)] = -2i DST(row i0)_k + 2 DST(row i0+1)_k.  The LDS sequence must be free.
template <typename T, int VPT>
__device__ __forceinline__ void g_dst_rows(const PinvArgs<T>& a, cplx<T>* c, const cplx<T>* tw, const T* in, int ld,
                                           int n, int nrow, int i0, bool valid, int tid, int nthr) {
    const int L = a.L;
    const bool two = i0 + 1 < nrow;
    cplx<T> v[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int p = tid + u * nthr;
        T x0 = T(0), x1 = T(0);
        if (valid) {
            // position p holds x_{p-1} (1 <= p <= n), -x_{L-1-p} (L-n <= p <= L-1), else 0
            const bool lo = (p >= 1 && p <= n);
            const bool hi = (p >= L - n);
            if (lo || hi) {
                const int m = lo ? p - 1 : L - 1 - p;
                const long long o = (long long)i0 * ld + m;
                x0 = in[o];
                if (two) x1 = in[o + ld];
                if (hi) {
                    x0 = -x0;
                    x1 = -x1;
                }
            }
        }
        v[u] = {x0, x1};
    }
    fft_x<T, VPT, false, true, false, true>(v, c, L, tw, tid, nthr);
}

// ---------------------------------------------------------------------------
// fused phases of the 2D tau-preconditioned CG (4 device-wide barriers per iteration)
//
// Row phases are organised per workgroup: its gpb groups transform 2 gpb adjacent rows (group g:
// rows ibase + 2g and ibase + 2g + 1, packed as one complex sequence).  Transposed intermediates
// (half spectra spec[k][i], sine-transform buffers t1/t2 [k][i], row stride ns) are written and
// read by the whole workgroup, thread (k, g) moving the two adjacent values of pair g, so that
// one wave covers 16 rows k with 2 gpb consecutive i each instead of one value per row.
// ---------------------------------------------------------------------------

// after each group's forward row FFT: spec[k][ibase + 2g (+1)] = half spectra of the pair's rows
template <typename T>
__device__ __forceinline__ void wg_write_spec(const PinvArgs<T>& a, const cplx<T>* cbase, int ibase, int gpb) {
    const int N = a.N, L = a.L, H = a.H, LP = lds_len(L);
    for (int idx = threadIdx.x; idx < H * gpb; idx += blockDim.x) {
        const int k = idx / gpb, g = idx - k * gpb;
        const int i = ibase + 2 * g;
        if (i >= N) continue;
        const cplx<T>* cg = cbase + (size_t)g * LP;
        const cplx<T> C = cg[lx(k)];
        const cplx<T> Cm = cg[lx((L - k) & (L - 1))];
        cplx<T>* dst = a.spec + (long long)k * a.ns + i;
        dst[0] = {T(0.5) * (C.x + Cm.x), T(0.5) * (C.y - Cm.y)};
        if (i + 1 < N) dst[1] = {T(0.5) * (C.y + Cm.y), T(0.5) * (Cm.x - C.x)};
    }
}

// after each group's sine-transform FFT (c[k+1] = -2i DST(row 2g) + 2 DST(row 2g+1)):
// out[k][ibase + 2g (+1)] = DST of the pair's rows at k, for k < nk and rows below nrow
// (row stride a.nt)
template <typename T>
__device__ __forceinline__ void wg_write_T(const PinvArgs<T>& a, const cplx<T>* cbase, T* out, int ibase, int gpb,
                                           int nk, int nrow) {
    const int LP = lds_len(a.L);
    for (int idx = threadIdx.x; idx < nk * gpb; idx += blockDim.x) {
        const int k = idx / gpb, g = idx - k * gpb;
        const int i = ibase + 2 * g;
        if (i >= nrow) continue;
        const cplx<T> C = cbase[(size_t)g * LP + lx(k + 1)];
        T* dst = out + (long long)k * a.nt + i;
        dst[0] = T(-0.5) * C.y;
        if (i + 1 < nrow) dst[1] = T(0.5) * C.x;
    }
}

// before the inverse row FFT: group g's sequence = Y0 + i Y1 over the full length, from the half
// spectra Y0, Y1 of its rows (Hermitian completion for k > L/2)
template <typename T>
__device__ __forceinline__ void wg_load_spec(const PinvArgs<T>& a, cplx<T>* cbase, int ibase, int gpb) {
    const int N = a.N, L = a.L, H = a.H, LP = lds_len(L);
    for (int idx = threadIdx.x; idx < H * gpb; idx += blockDim.x) {
        const int k = idx / gpb, g = idx - k * gpb;
        const int i = ibase + 2 * g;
        cplx<T> Y0 = {T(0), T(0)}, Y1 = {T(0), T(0)};
        if (i < N) {
            const cplx<T>* src = a.spec + (long long)k * a.ns + i;
            Y0 = src[0];
            if (i + 1 < N) Y1 = src[1];
        }
        cplx<T>* cg = cbase + (size_t)g * LP;
        cg[lx(k)] = {Y0.x - Y1.y, Y0.y + Y1.x};
        if (k > 0 && k < H - 1) cg[lx(L - k)] = {Y0.x + Y1.y, Y1.x - Y0.y};
    }
}

// pass B: rows k0 = kbase + 2g (+1) of t1 hold (S r)^T rows; a DST over i gives Y = S r S (up to
// scale), Y is scaled by scale/(sigma + c tau) and transformed again into t2 = S Yhat (transposed).
// (r, z) = (r, M^{-1} r) = scale * sum Y^2/(sigma + c tau) is accumulated in rz.  tau is stored
// [k2][k1], so the eigenvalues for rows k0, k0 + 1 are two contiguous rows.
template <typename T, int VPT>
__device__ __forceinline__ void wg_pass_B(const PinvArgs<T>& a, cplx<T>* cbase, cplx<T>* c, const cplx<T>* tw, int kbase, int grp,
                          int gpb, T sig, T cc, T scale, int tid, int nthr, T& rz) {
    // rows k0, k0 + 1 of t1 (first-transform frequencies, Nt of them) hold N values each
    const int N = a.N, Nt = a.Nt;
    const int k0 = kbase + 2 * grp;
    const bool valid = k0 < Nt;
    const bool two = k0 + 1 < Nt;
    constexpr bool PREF = VPT <= 8;  // prefetch the epilogue operands before the transform
    constexpr int VH = VPT / 2;      // k1 < Nt < L/2 = VH * nthr
    T tv0[VH], tv1[VH];
    auto load_tau = [&](int u) {
        const int k1 = tid + u * nthr;
        tv0[u] = tv1[u] = T(1);
        if (valid && k1 < Nt) {
            tv0[u] = a.tau[(long long)k0 * Nt + k1];
            if (two) tv1[u] = a.tau[(long long)(k0 + 1) * Nt + k1];
        }
    };
    if constexpr (PREF) {
#pragma unroll
        for (int u = 0; u < VH; ++u) load_tau(u);
    }
    g_dst_rows<T, VPT>(a, c, tw, a.t1, a.nt, N, Nt, k0, valid, tid, nthr);
    T hv0[VH], hv1[VH];
#pragma unroll
    for (int u = 0; u < VH; ++u) {
        const int k1 = tid + u * nthr;
        hv0[u] = hv1[u] = T(0);
        if constexpr (!PREF) load_tau(u);
        if (valid && k1 < Nt) {
            const cplx<T> C = c[lx(k1 + 1)];
            const T y0 = T(-0.5) * C.y, y1 = T(0.5) * C.x;
            hv0[u] = y0 * scale / (sig + cc * tv0[u]);
            rz += y0 * hv0[u];
            if (two) {
                hv1[u] = y1 * scale / (sig + cc * tv1[u]);
                rz += y1 * hv1[u];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < VH; ++u) {
        const int k1 = tid + u * nthr;
        if (k1 < Nt) {
            c[lx(k1 + 1)] = {hv0[u], hv1[u]};
            c[lx(a.L - k1 - 1)] = {-hv0[u], -hv1[u]};
        }
    }
    if (tid == 0) {
        c[lx(0)] = {T(0), T(0)};
        c[lx(Nt + 1)] = {T(0), T(0)};
    }
    __syncthreads();
    fft_lds<T, VPT, false, true>(c, a.L, tw, tid, nthr);
    // back in space along the columns: rows i < N of t2, columns k0, k0 + 1
    wg_write_T(a, cbase, a.t2, kbase, gpb, N, Nt);
    __syncthreads();
}

// pass D of z = M^{-1} r on rows (i0, i1) of t2 (z rows), then p = z + beta p, (p, dg p), and the
// forward row transform of the new p rows into the half spectra.
template <typename T, int VPT>
__device__ __forceinline__ void wg_pass_DF(const PinvArgs<T>& a, cplx<T>* cbase, cplx<T>* c, const cplx<T>* tw, int ibase, int grp,
                           int gpb, T beta, const T* dg, int tid, int nthr, T& pdp) {
    const int N = a.N, L = a.L;
    const int i0 = ibase + 2 * grp;
    const bool valid = i0 < N;
    const bool two = i0 + 1 < N;
    constexpr bool PREF = VPT <= 8;  // prefetch the epilogue operands before the transform
    constexpr int VH = VPT / 2;      // m < N < L/2 = VH * nthr
    T pold0[VH], pold1[VH], d0[VH], d1[VH];
    auto load_pd = [&](int u) {
        const int m = tid + u * nthr;
        pold0[u] = pold1[u] = d0[u] = d1[u] = T(0);
        if (valid && m < N) {
            const long long o0 = (long long)i0 * N + m;
            if (beta != T(0)) {
                pold0[u] = a.p[o0];
                if (two) pold1[u] = a.p[o0 + N];
            }
            if (dg) {
                d0[u] = dg[o0];
                if (two) d1[u] = dg[o0 + N];
            }
        }
    };
    if constexpr (PREF) {
#pragma unroll
        for (int u = 0; u < VH; ++u) load_pd(u);
    }
    g_dst_rows<T, VPT>(a, c, tw, a.t2, a.nt, a.Nt, N, i0, valid, tid, nthr);
    T pn0[VH], pn1[VH];
#pragma unroll
    for (int u = 0; u < VH; ++u) {
        const int m = tid + u * nthr;
        pn0[u] = pn1[u] = T(0);
        if constexpr (!PREF) load_pd(u);
        if (valid && m < N) {
            const cplx<T> C = c[lx(m + 1)];
            pn0[u] = T(-0.5) * C.y + beta * pold0[u];
            if (two) pn1[u] = T(0.5) * C.x + beta * pold1[u];
            pdp += d0[u] * pn0[u] * pn0[u] + d1[u] * pn1[u] * pn1[u];
            const long long o0 = (long long)i0 * N + m;
            a.p[o0] = pn0[u];
            if (two) a.p[o0 + N] = pn1[u];
        }
    }
    cplx<T> v[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) v[u] = (u < VH) ? cplx<T>{pn0[u], pn1[u]} : cplx<T>{T(0), T(0)};
    __syncthreads();  // every thread has read its sine-transform values: the sequence is free
    fft_x<T, VPT, false, true, false, true>(v, c, L, tw, tid, nthr);
    wg_write_spec(a, cbase, ibase, gpb);
    __syncthreads();
}

// column pass of B p with (p, B p) = sum |V|^2 lambda/L^2 over the full spectrum (the half spectrum
// counted twice except k2 = 0 and L/2)
template <typename T, int VPT>
__device__ __forceinline__ void g_cols_pbp(const PinvArgs<T>& a, cplx<T>* c, const cplx<T>* tw, int k2, bool valid, int tid, int nthr,
                           T& pbp) {
    // both transforms register-resident: thread tid holds positions tid + u nthr throughout
    const int N = a.N, L = a.L;
    cplx<T>* row = a.spec + (long long)k2 * a.ns;
    const T* sy = a.sym + (long long)k2 * L;
    constexpr int VH = VPT / 2;  // i < N < L/2 = VH * nthr
    T sv[VPT];
    cplx<T> v[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int i = tid + u * nthr;
        v[u] = (u < VH && valid && i < N) ? row[i] : cplx<T>{T(0), T(0)};
        sv[u] = valid ? sy[i] : T(0);
    }
    fft_x<T, VPT, false, true, true, true>(v, c, L, tw, tid, nthr);
    const T wk = (k2 == 0 || 2 * k2 == L) ? T(1) : T(2);
    T acc = T(0);
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        acc += (v[u].x * v[u].x + v[u].y * v[u].y) * sv[u];
        v[u] = {v[u].x * sv[u], v[u].y * sv[u]};
    }
    pbp += wk * acc;
    fft_x<T, VPT, true, true, true, true>(v, c, L, tw, tid, nthr);
    if (valid) {
#pragma unroll
        for (int u = 0; u < VH; ++u) {
            const int i = tid + u * nthr;
            if (i < N) row[i] = v[u];
        }
    }
}

// inverse row transform -> u = B p rows; q = dg p + c u; r -= alpha q; x += alpha p; (r, r);
// then pass A (DST of the new r rows into t1)
template <typename T, int VPT>
__device__ __forceinline__ void wg_pass_IUA(const PinvArgs<T>& a, cplx<T>* cbase, cplx<T>* c, const cplx<T>* tw, int ibase, int grp,
                            int gpb, const T* dg, T cc, T alpha, int tid, int nthr, T& rr) {
    const int N = a.N, L = a.L;
    const int i0 = ibase + 2 * grp;
    const bool valid = i0 < N;
    const bool two = i0 + 1 < N;
    constexpr bool PREF = VPT <= 8;  // prefetch the epilogue operands before the transform
    constexpr int VH = VPT / 2;      // m < N < L/2 = VH * nthr
    T p0[VH], p1[VH], d0[VH], d1[VH], r0[VH], r1[VH], x0[VH], x1[VH];
    auto load_prx = [&](int u) {
        const int m = tid + u * nthr;
        p0[u] = p1[u] = d0[u] = d1[u] = r0[u] = r1[u] = x0[u] = x1[u] = T(0);
        if (valid && m < N) {
            const long long o0 = (long long)i0 * N + m;
            p0[u] = a.p[o0];
            r0[u] = a.r[o0];
            x0[u] = a.x[o0];
            if (dg) d0[u] = dg[o0];
            if (two) {
                p1[u] = a.p[o0 + N];
                r1[u] = a.r[o0 + N];
                x1[u] = a.x[o0 + N];
                if (dg) d1[u] = dg[o0 + N];
            }
        }
    };
    if constexpr (PREF) {
#pragma unroll
        for (int u = 0; u < VH; ++u) load_prx(u);
    }
    wg_load_spec(a, cbase, ibase, gpb);
    __syncthreads();
    cplx<T> bp[VPT];
    fft_x<T, VPT, true, false, true, true>(bp, c, L, tw, tid, nthr);  // B p rows left in registers
#pragma unroll
    for (int u = 0; u < VH; ++u) {
        const int m = tid + u * nthr;
        if constexpr (!PREF) load_prx(u);
        const cplx<T> uu = bp[u];
        if (valid && m < N) {
            const T q0 = d0[u] * p0[u] + cc * uu.x;
            r0[u] -= alpha * q0;
            x0[u] += alpha * p0[u];
            const long long o0 = (long long)i0 * N + m;
            a.r[o0] = r0[u];
            a.x[o0] = x0[u];
            rr += r0[u] * r0[u];
            if (two) {
                const T q1 = d1[u] * p1[u] + cc * uu.y;
                r1[u] -= alpha * q1;
                x1[u] += alpha * p1[u];
                a.r[o0 + N] = r1[u];
                a.x[o0 + N] = x1[u];
                rr += r1[u] * r1[u];
            } else {
                r1[u] = T(0);
            }
        } else {
            r0[u] = r1[u] = T(0);
        }
    }
    // pass A on the updated rows: odd extension (zero for m >= N, so the padded entries and the
    // middle position L/2), FFT, DST rows -> t1 (transposed); the sequence is free (the inverse
    // transform left its output in registers)
#pragma unroll
    for (int u = 0; u < VH; ++u) {
        const int m = tid + u * nthr;
        c[lx(m + 1)] = {r0[u], r1[u]};
        c[lx(L - m - 1)] = {-r0[u], -r1[u]};
    }
    if (tid == 0) c[lx(0)] = {T(0), T(0)};
    __syncthreads();
    fft_lds<T, VPT, false, true>(c, L, tw, tid, nthr);
    wg_write_T(a, cbase, a.t1, ibase, gpb, a.Nt, N);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// segment kernel: steps [sa, sb)
// ---------------------------------------------------------------------------
// twiddles live in LDS beside the sequences unless that exceeds the 160 KB of a CU (FP64, L = 8192)
template <typename T>
__host__ __device__ constexpr bool tw_in_lds(int vpt) { return !(vpt == 32 && sizeof(T) == 8); }

constexpr int kSegBlock = 256;  // workgroup size of the 2D segment kernel (1D: one transform group)

// kernel variants: the 1D problem, the 2D problem with the diagonal preconditioner, and the 2D
// problem with the sine-transform (tau) preconditioner and its fused CG phases
enum SegMode : int { SEG_1D = 0, SEG_2D_DIAG = 1, SEG_2D_TAU = 2 };

// row stride of the transposed 2D intermediates: N rounded up to 16 values, so that the rows of
// spec (16-byte complex FP64) start on 256-byte boundaries
__host__ __device__ constexpr int spec_stride(int N) { return (N + 15) & ~15; }

// LC > 0: the transform length is the compile-time constant LC (2D sine-transform path, where
// L = 2(N + 1)); LC = 0: lengths are taken from the arguments
// TB: the tau-block form (each block solved by one application of its frozen-coefficient tau
// matrix, from zero; 2D tau path only)
template <typename T, int VPT, int MODE, int LC, bool TB>
__device__ __forceinline__ void segment_run(PinvArgs<T> a, int sa, int sb) {
    static_assert(LC == 0 || MODE == SEG_2D_TAU, "a fixed length is provided for the 2D tau path only");
    static_assert(!TB || MODE == SEG_2D_TAU, "the tau-block form runs on the 2D tau path only");
    if constexpr (LC > 0) {
        a.d = 2;
        a.L = LC;
        a.N = LC / 2 - 1;
        a.Nt = LC / 2 - 1;
        a.H = LC / 2 + 1;
        a.Nd = (long long)(LC / 2 - 1) * (LC / 2 - 1);
        a.ns = spec_stride(LC / 2 - 1);
        a.nt = a.ns;
    }
    extern __shared__ unsigned char smem_raw[];
    __shared__ double red[kSegBlock / 64 * 2];
    __shared__ double tot[kNPart];
    // the history weights e_0 .. e_kHB and the shifts sigma_s of the segment's steps, read once per
    // launch (a read from global memory after every device-wide synchronisation misses the caches)
    __shared__ T s_e[kHB + 1];
    __shared__ double s_sig[kHB];
    constexpr bool TWL = tw_in_lds<T>(VPT);
    constexpr bool TAU2 = (MODE == SEG_2D_TAU);
    constexpr bool two_d = (MODE != SEG_1D);
    const int nthr = a.L / VPT;             // threads per transform group
    const int gpb = blockDim.x / nthr;      // groups per workgroup (1 for d = 1)
    const int grp = threadIdx.x / nthr;
    const int tid = threadIdx.x - grp * nthr;
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int twn = TWL ? a.L : 0;  // twiddles first (when in LDS), then the sequences
    cplx<T>* cbase = lds + twn;     // the groups' sequences
    cplx<T>* c = cbase + (size_t)grp * lds_len(a.L);
    // near-history ring (a.ring): slot i holds y_{sa+i} of the thread's points, [i][u][q][thread]
    T* ring = reinterpret_cast<T*>(cbase + (size_t)gpb * lds_len(a.L));
    for (int k = threadIdx.x; k < twn; k += blockDim.x) lds[k] = a.tw[k];
    for (int k = threadIdx.x; k <= kHB; k += blockDim.x) s_e[k] = (a.epad + kEpad)[k];
    for (int k = threadIdx.x; k < kHB; k += blockDim.x) s_sig[k] = (sa + k < a.M) ? a.sigma[sa + k] : 0.0;
    const cplx<T>* twl = TWL ? lds : a.tw;
    __syncthreads();
    const int NG = a.vg * gpb;         // groups in the grid
    const int gg = a.vb * gpb + grp;  // this group's index
    const long long gtid = (long long)a.vb * blockDim.x + threadIdx.x;
    const long long gthreads = (long long)a.vg * blockDim.x;
    const int N = a.N;
    const long long Nd = a.Nd;
    const int M = a.M;
    const int NP = two_d ? (N + 1) / 2 : 1;  // row pairs (2D)
    const int NR = (NP + NG - 1) / NG;       // rounds over row pairs
    const int NC = (a.H + NG - 1) / NG;      // rounds over spectral rows
    const int NRB = ((a.Nt + 1) / 2 + NG - 1) / NG;  // rounds over frequency pairs of the sine transform
    const T scale = two_d ? T(4.0 / ((double)(a.Nt + 1) * (a.Nt + 1))) : T(2.0 / (a.Nt + 1));
    unsigned ph = 0;  // phase of the device-wide synchronisation (phase_sync)
    auto sync_bar = [&]() { phase_barrier(a.part, a.bar, a.bar_ticks, red, tot, ph, a.vb, a.vg); };
    long long total_it = 0;

    for (int s = sa; s < sb; ++s) {
        const bool lastrow = (s == M);
        const T* dg = lastrow ? nullptr : a.dg + (long long)s * Nd;
        const T cc = lastrow ? T(1) : a.ct;
        const T sig = lastrow ? T(0) : T(s_sig[s - sa]);

        // z = M^{-1} r and (r, z) for the 1D tau and the diagonal preconditioners (the 2D tau
        // preconditioner has its own fused loop below), optionally after the CG update
        auto prec_A = [&](bool upd, T alpha) {
            T rr = T(0), rzl = T(0);
            if (a.use_tau) {
                const bool act = gg == 0;
                g_dst_load<T, VPT>(a, c, twl, a.r, N, 0, act, tid, nthr, upd, alpha, rr);
                // sine-transform coefficients k < Nt (the transform size; Nt >= N)
                const int Nt = a.Nt;
                T hv[VPT], tv[VPT], rv[VPT];
#pragma unroll
                for (int u = 0; u < VPT; ++u) {
                    const int k = tid + u * nthr;
                    tv[u] = (k < Nt) ? a.tau[k] : T(1);
                    rv[u] = (act && k < N) ? a.r[k] : T(0);
                }
#pragma unroll
                for (int u = 0; u < VPT; ++u) {
                    const int k = tid + u * nthr;
                    hv[u] = (k < Nt) ? T(-0.5) * c[lx(k + 1)].y * scale / (sig + cc * tv[u]) : T(0);
                }
                __syncthreads();
#pragma unroll
                for (int u = 0; u < VPT; ++u) {
                    const int k = tid + u * nthr;
                    if (k < Nt) {
                        c[lx(k + 1)] = {hv[u], T(0)};
                        c[lx(a.L - k - 1)] = {-hv[u], T(0)};
                    }
                }
                if (tid == 0) {
                    c[lx(0)] = {T(0), T(0)};
                    c[lx(Nt + 1)] = {T(0), T(0)};
                }
                __syncthreads();
                fft_lds<T, VPT, false, true>(c, a.L, twl, tid, nthr);
                if (act) {
#pragma unroll
                    for (int u = 0; u < VPT; ++u) {
                        const int k = tid + u * nthr;
                        if (k < N) {
                            const T zv = T(-0.5) * c[lx(k + 1)].y;
                            a.zz[k] = zv;
                            rzl += rv[u] * zv;
                        }
                    }
                }
                __syncthreads();
            } else {
                for (long long j = gtid; j < Nd; j += gthreads) {
                    T rv = a.r[j];
                    const T qv = upd ? a.q[j] : T(0);
                    const T xv = upd ? a.x[j] : T(0);
                    const T pv = upd ? a.p[j] : T(0);
                    const T dv = dg ? dg[j] : T(0);
                    if (upd) {
                        rv -= alpha * qv;
                        a.x[j] = xv + alpha * pv;
                        a.r[j] = rv;
                        rr += rv * rv;
                    }
                    const T zv = rv / (dv + cc * a.a0);
                    a.zz[j] = zv;
                    rzl += rv * zv;
                }
            }
            if (upd) {
                const int sl[2] = {SL_RR, SL_RZ};
                const T vv[2] = {rr, rzl};
                phase_sync<2, true, -1>(a.part, a.bar, a.bar_ticks, sl, vv, red, tot, ph, a.vb, a.vg);
            } else {
                const int sl[1] = {SL_RZ};
                const T vv[1] = {rzl};
                phase_sync<1, true, -1>(a.part, a.bar, a.bar_ticks, sl, vv, red, tot, ph, a.vb, a.vg);
            }
        };

        // ---------------- E: finish step s-1, history, rhs, warm start, r0 ----------------
        // For point j: y_{s-1} = x is stored, B y_{s-1} is recovered from the residual identity, the
        // history term and the right-hand side of block row s are formed, the warm start x0 (linear
        // extrapolation in time) and r0 = rhs - A_s x0 are stored; returns r0 and adds to (r, r), (b, b).
        const int nnear = s - sa;  // near-history terms m in [sa, s)
        struct EIn {
            T xv, rhs_o, r_o, dgp, bxb, bxb2, ym2, ym3, zo, g2o, dgo, hn;
        };
        // weights of the near-history terms y_{sa+i}, i < kHB, of this step (zero for absent terms),
        // read once per step so that no load of a point waits on a weight
        T ew[kNear];
#pragma unroll
        for (int i = 0; i < kNear; ++i) ew[i] = (!lastrow && i + 1 < nnear) ? s_e[s - sa - i] : T(0);
        const T e1 = (nnear >= 1) ? s_e[1] : T(0);  // weight of y_{s-1} when it is a near term
        // loads of point j (no stores, so that the loads of several points can be in flight together);
        // hn = sum over the near-history terms m in [sa, s-1) of e_{s-m} y_m, read from the LDS ring when
        // the thread keeps its points' earlier solutions there (a.ring), else from y
        // (u, q): the point's column round and row within the thread's row pair (the ring's index), or
        // q < 0 for the grid-stride form, which does not use the ring
        // the common step (s > 0, not the last block row, no extrapolation; either sweep): only the
        // six values it uses are loaded, so that the loads of all of a thread's points stay within
        // the count of memory operations in flight that the hardware tracks
        auto e_load_lean = [&](long long j, int u, int q) -> EIn {
            EIn v;
            v.xv = a.x[j];
            v.rhs_o = a.rhs[j];
            v.r_o = a.r[j];
            v.dgp = a.dg[(long long)(s - 1) * Nd + j];
            v.zo = a.hacc[(long long)(s - sa) * Nd + j];
            v.dgo = dg[j];
            v.bxb = v.bxb2 = v.ym2 = v.ym3 = T(0);
            v.g2o = T(1);
            T yv[kNear];
#pragma unroll
            for (int i = 0; i < kNear; ++i) yv[i] = ring[((i * (VPT / 2) + u) * 2 + q) * (int)blockDim.x + threadIdx.x];
#pragma unroll
            for (int i = 0; i < kNear; ++i) yv[i] = (i + 1 < nnear) ? yv[i] : T(0);
            T hn = T(0);
#pragma unroll
            for (int i = 0; i < kNear; ++i) hn += ew[i] * yv[i];
            v.hn = hn;
            return v;
        };
        auto e_load = [&](long long j, int u, int q) -> EIn {
            // Every load is issued unconditionally from an address inside its array (an unused value
            // comes from x, or from a clamped slice) and the value is selected afterwards: a load
            // under a condition with a zero default makes the compiler wait for every load in flight
            // before it writes the default into the load's register, which serialises the points.
            EIn v;
            const bool ext = (s >= 2 && !lastrow && a.extrap && !TB);
            const bool ext2 = (s >= 3 && !lastrow && a.extrap == 2 && !TB);
            const T xl = a.x[j], rhsl = a.rhs[j], rl = a.r[j];
            const T dgpl = a.dg[(long long)max(s - 1, 0) * Nd + j];
            const T bxbl = (ext ? a.bxb : a.x)[j];
            const T ym2l = ext ? a.y[(long long)max(s - 2, 0) * Nd + j] : a.x[j];
            const T ym3l = ext2 ? a.y[(long long)max(s - 3, 0) * Nd + j] : a.x[j];
            const T bxb2l = (ext2 ? a.bxb2 : a.x)[j];
            // s < M: w_s (far history folded in) and dg_s = gamma1_s/gamma2_s (e_0 = 1);
            // s = M: z_M and gamma2_{M-1}
            const T zol = (lastrow ? a.z + (long long)M * Nd : a.hacc + (long long)(s - sa) * Nd)[j];
            const T g2l = (lastrow ? a.g2 + (long long)(M - 1) * Nd : a.x)[j];
            const T dgol = (dg ? dg : a.dg)[j];
            // y_m for m = sa + i < s - 1 (y_{s-1} is xv), from the ring or from y (slice clamped)
            const bool lring = a.ring && q >= 0;
            T yv[kNear];
#pragma unroll
            for (int i = 0; i < kNear; ++i)
                yv[i] = lring ? ring[((i * (VPT / 2) + u) * 2 + q) * (int)blockDim.x + threadIdx.x]
                              : a.y[(long long)min(sa + i, M - 1) * Nd + j];
            v.xv = (s > 0) ? xl : T(0);
            v.rhs_o = (s > 0) ? rhsl : T(0);
            v.r_o = (s > 0) ? rl : T(0);
            v.dgp = (s > 0) ? dgpl : T(0);
            v.bxb = ext ? bxbl : T(0);
            v.ym2 = ext ? ym2l : T(0);
            v.ym3 = ext2 ? ym3l : T(0);
            v.bxb2 = ext2 ? bxb2l : T(0);
            v.zo = zol;
            v.g2o = lastrow ? g2l : T(1);
            v.dgo = dg ? dgol : T(0);
#pragma unroll
            for (int i = 0; i < kNear; ++i) yv[i] = (!lastrow && i + 1 < nnear) ? yv[i] : T(0);
            if (a.adj && !lring) {
                // transposed sweep: each earlier step's term carries its own weight dg_m (the ring
                // holds the products already)
#pragma unroll
                for (int i = 0; i < kNear; ++i)
                    if (!lastrow && i + 1 < nnear) yv[i] *= a.dg[(long long)(sa + i) * Nd + j];
            }
            T hn = T(0);
#pragma unroll
            for (int i = 0; i < kNear; ++i) hn += ew[i] * yv[i];
            v.hn = hn;
            return v;
        };
        // the values of point j (no memory access), then its stores (e_write): a round forms all its
        // points before it stores any, so that no store waits behind the loads of a later point
        struct EOut {
            T yprev, bxprev, bxb_old, rhs, x0, rv, dgp;
        };
        auto e_form = [&](const EIn& v) -> EOut {
            const bool ext = (s >= 2 && !lastrow && a.extrap && !TB);
            const bool ext2 = (s >= 3 && !lastrow && a.extrap == 2 && !TB);
            const T yprev = v.xv;
            const T bxprev = (s > 0) ? (v.rhs_o - v.r_o - v.dgp * yprev) / a.ct : T(0);  // B y_{s-1}
            const T hn = v.hn;
            T rhs, x0 = T(0), bx0 = T(0);
            if (lastrow) {
                rhs = (v.zo - yprev) / (a.cf * v.g2o);
            } else if (a.adj) {
                rhs = v.zo - (hn + e1 * v.dgp * yprev);  // transposed sweep: weights of the earlier steps
            } else {
                const T h = hn + e1 * yprev;
                rhs = v.zo - v.dgo * h;
                if (s >= 1 && !TB) {
                    // linear (or, extrap = 2, quadratic) extrapolation in time of y and B y
                    if (ext2) {
                        x0 = T(3) * (yprev - v.ym2) + v.ym3;
                        bx0 = T(3) * (bxprev - v.bxb) + v.bxb2;
                    } else {
                        const T th = (a.extrap == 3) ? T(0.5) : T(1);  // 3: half the linear step
                        x0 = ext ? yprev + th * (yprev - v.ym2) : yprev;
                        bx0 = ext ? bxprev + th * (bxprev - v.bxb) : bxprev;
                    }
                }
            }
            const T rv = rhs - (v.dgo * x0 + cc * bx0);
            return EOut{yprev, bxprev, v.bxb, rhs, x0, rv, v.dgp};
        };
        auto e_write = [&](long long j, const EOut& o, T& rr, T& bb, int u, int q) {
            if (s > 0) a.y[(long long)(s - 1) * Nd + j] = o.yprev;
            // the transposed sweep keeps dg_{s-1} y_{s-1}, the term its near-history sum weighs
            if (a.ring && q >= 0 && s > sa && s - 1 - sa < kNear)
                ring[(((s - 1 - sa) * (VPT / 2) + u) * 2 + q) * (int)blockDim.x + threadIdx.x] =
                    a.adj ? o.yprev * o.dgp : o.yprev;
            if (s >= 1 && !lastrow && a.extrap && !TB) {
                a.bxb[j] = o.bxprev;  // B y_{s-1} is "B y_{s-2}" next step
                if (a.extrap == 2) a.bxb2[j] = o.bxb_old;  // and B y_{s-2} is "B y_{s-3}"
            }
            a.rhs[j] = o.rhs;
            a.x[j] = o.x0;
            a.r[j] = o.rv;
            rr += o.rv * o.rv;
            bb += o.rhs * o.rhs;
        };
        {
            T rr = T(0), bb = T(0);
            if constexpr (TAU2) {
                // row ownership (group: rows i0, i0 + 1), fused with pass A of z0 = M^{-1} r0: the new
                // residual rows are sine-transformed into t1 right away
                for (int rd = 0; rd < NR; ++rd) {
                    const int ibase = 2 * (rd * NG + a.vb * gpb);
                    const int i0 = ibase + 2 * grp;
                    const bool valid = i0 < N;
                    const bool two = i0 + 1 < N;
                    // points (i0 + q, m = tid + u nthr), m < N < L/2: the loads of EB columns u (both
                    // rows) are issued together, then the values are formed and stored
                    constexpr int VH = VPT / 2;
                    // EB columns per round: all of them when the near history comes from the ring (the
                    // loads of a round then stay within the count of memory operations in flight that
                    // the hardware tracks), else two
                    auto e_rounds = [&](auto ebc, auto leanc) {
                    constexpr int EB = decltype(ebc)::value;
                    constexpr bool LEAN = decltype(leanc)::value;
#pragma unroll 1
                    for (int u0 = 0; u0 < VH; u0 += EB) {
                        EIn v[EB][2];
#pragma unroll
                        for (int du = 0; du < EB; ++du) {
                            const int m = tid + (u0 + du) * nthr;
                            if (valid && m < N) {
                                const long long j0 = (long long)i0 * N + m;
                                if constexpr (LEAN) {
                                    v[du][0] = e_load_lean(j0, u0 + du, 0);
                                    if (two) v[du][1] = e_load_lean(j0 + N, u0 + du, 1);
                                } else {
                                    v[du][0] = e_load(j0, u0 + du, 0);
                                    if (two) v[du][1] = e_load(j0 + N, u0 + du, 1);
                                }
                            }
                        }
                        EOut o[EB][2];
#pragma unroll
                        for (int du = 0; du < EB; ++du) {
                            const int m = tid + (u0 + du) * nthr;
                            if (valid && m < N) {
                                o[du][0] = e_form(v[du][0]);
                                if (two) o[du][1] = e_form(v[du][1]);
                            }
                        }
#pragma unroll
                        for (int du = 0; du < EB; ++du) {
                            // m < L/2: zero past the data (padded entries, position L/2)
                            const int m = tid + (u0 + du) * nthr;
                            T r0 = T(0), r1 = T(0);
                            if (valid && m < N) {
                                const long long j0 = (long long)i0 * N + m;
                                e_write(j0, o[du][0], rr, bb, u0 + du, 0);
                                r0 = o[du][0].rv;
                                if (two) {
                                    e_write(j0 + N, o[du][1], rr, bb, u0 + du, 1);
                                    r1 = o[du][1].rv;
                                }
                            }
                            c[lx(m + 1)] = {r0, r1};
                            c[lx(a.L - m - 1)] = {-r0, -r1};
                        }
                    }
                    };
                    const bool lean = a.ring && s > 0 && !lastrow && !(a.extrap && s >= 2 && !TB);
                    if (lean) e_rounds(std::integral_constant<int, VH>{}, std::true_type{});
                    else if (a.ring) e_rounds(std::integral_constant<int, VH>{}, std::false_type{});
                    else e_rounds(std::integral_constant<int, (VH >= 2 ? 2 : 1)>{}, std::false_type{});
                    if (tid == 0) c[lx(0)] = {T(0), T(0)};
                    __syncthreads();
                    fft_lds<T, VPT, false, true>(c, a.L, twl, tid, nthr);
                    wg_write_T(a, cbase, a.t1, ibase, gpb, a.Nt, N);
                    __syncthreads();
                }
            } else {
                for (long long j = gtid; j < Nd; j += gthreads) e_write(j, e_form(e_load(j, 0, -1)), rr, bb, 0, -1);
            }
            {
                const int sl[2] = {SL_RR, SL_BB};
                const T vv[2] = {rr, bb};
                phase_sync<2, true, -1>(a.part, a.bar, a.bar_ticks, sl, vv, red, tot, ph, a.vb, a.vg);
            }
        }
        const double bbt = tot[SL_BB];
        double rrt = tot[SL_RR];
        if (!(bbt > 0.0)) {
            // zero right-hand side: the solution is zero
            for (long long j = gtid; j < Nd; j += gthreads) {
                a.x[j] = T(0);
                a.r[j] = T(0);
            }
            sync_bar();
            continue;
        }
        if constexpr (TAU2) {
            if constexpr (TB) {
                // y_s = M_s^{-1} rhs_s: pass B, then the last sine transform of each row pair straight
                // into x.  The next step's phase E reads these points in the same thread, so no
                // device-wide barrier follows.
                T rzl = T(0);
                for (int rd = 0; rd < NRB; ++rd) {
                    const int kbase = 2 * (rd * NG + a.vb * gpb);
                    wg_pass_B<T, VPT>(a, cbase, c, twl, kbase, grp, gpb, sig, cc, scale, tid, nthr, rzl);
                }
                sync_bar();
                for (int rd = 0; rd < NR; ++rd) {
                    const int ibase = 2 * (rd * NG + a.vb * gpb);
                    const int i0 = ibase + 2 * grp;
                    const bool valid = i0 < N;
                    g_dst_rows<T, VPT>(a, c, twl, a.t2, a.nt, a.Nt, N, i0, valid, tid, nthr);
#pragma unroll
                    for (int u = 0; u < VPT / 2; ++u) {
                        const int m = tid + u * nthr;
                        if (valid && m < N) {
                            const cplx<T> C = c[lx(m + 1)];
                            const long long o0 = (long long)i0 * N + m;
                            a.x[o0] = T(-0.5) * C.y;
                            if (i0 + 1 < N) a.x[o0 + N] = T(0.5) * C.x;
                        }
                    }
                    __syncthreads();  // the sequences are reused
                }
                continue;
            }
        }
        if (rrt <= a.tol2 * bbt) continue;  // the warm start already meets the tolerance

        // ---------------- preconditioned CG ----------------
        if constexpr (TAU2) {
            // z0 = M^{-1} r0: pass A ran with phase E; pass B (with (r, z))
            {
                T rzl = T(0);
                for (int rd = 0; rd < NRB; ++rd) {
                    const int kbase = 2 * (rd * NG + a.vb * gpb);
                    wg_pass_B<T, VPT>(a, cbase, c, twl, kbase, grp, gpb, sig, cc, scale, tid, nthr, rzl);
                }
                const int sl[1] = {SL_RZ};
                const T vv[1] = {rzl};
                phase_sync<1, true, -1>(a.part, a.bar, a.bar_ticks, sl, vv, red, tot, ph, a.vb, a.vg);
            }
            double rz = tot[SL_RZ];
            T beta = T(0);
            int it = 0;
            while (true) {
                T pdp = T(0), pbp = T(0), rr = T(0);
                for (int rd = 0; rd < NR; ++rd) {
                    const int ibase = 2 * (rd * NG + a.vb * gpb);
                    wg_pass_DF<T, VPT>(a, cbase, c, twl, ibase, grp, gpb, beta, dg, tid, nthr, pdp);
                }
                {
                    const int sl[1] = {SL_PD};
                    const T vv[1] = {pdp};
                    phase_sync<1, false, -1>(a.part, a.bar, a.bar_ticks, sl, vv, red, tot, ph, a.vb, a.vg);
                }
                for (int rd = 0; rd < NC; ++rd) {
                    const int k2 = rd * NG + gg;
                    g_cols_pbp<T, VPT>(a, c, twl, k2, k2 < a.H, tid, nthr, pbp);
                }
                {
                    const int sl[1] = {SL_PB};
                    const T vv[1] = {pbp};
                    phase_sync<1, true, SL_PD>(a.part, a.bar, a.bar_ticks, sl, vv, red, tot, ph, a.vb, a.vg);
                }
                const double pqt = tot[SL_PD] + (double)cc * tot[SL_PB];
                const T alpha = T(pqt != 0.0 ? rz / pqt : 0.0);
                for (int rd = 0; rd < NR; ++rd) {
                    const int ibase = 2 * (rd * NG + a.vb * gpb);
                    wg_pass_IUA<T, VPT>(a, cbase, c, twl, ibase, grp, gpb, dg, cc, alpha, tid, nthr, rr);
                }
                {
                    const int sl[1] = {SL_RR};
                    const T vv[1] = {rr};
                    phase_sync<1, true, -1>(a.part, a.bar, a.bar_ticks, sl, vv, red, tot, ph, a.vb, a.vg);
                }
                ++it;
                rrt = tot[SL_RR];
                if (rrt <= a.tol2 * bbt || it >= a.maxit || !(rrt == rrt)) break;
                T rzl = T(0);
                for (int rd = 0; rd < NRB; ++rd) {
                    const int kbase = 2 * (rd * NG + a.vb * gpb);
                    wg_pass_B<T, VPT>(a, cbase, c, twl, kbase, grp, gpb, sig, cc, scale, tid, nthr, rzl);
                }
                {
                    const int sl[1] = {SL_RZ};
                    const T vv[1] = {rzl};
                    phase_sync<1, true, -1>(a.part, a.bar, a.bar_ticks, sl, vv, red, tot, ph, a.vb, a.vg);
                }
                const double rz_new = tot[SL_RZ];
                beta = T(rz != 0.0 ? rz_new / rz : 0.0);
                rz = rz_new;
            }
            total_it += it;
            continue;
        } else {
        prec_A(false, T(0));
        double rz = tot[SL_RZ];
        T beta = T(0);
        int it = 0;
        while (true) {
            // q = A_s p with p = z + beta p ; (p, q)
            T pq = T(0);
            if constexpr (two_d) {
                for (int rd = 0; rd < NR; ++rd) {
                    const int pr = rd * NG + gg;
                    g_rows_fwd<T, VPT>(a, c, twl, pr, pr < NP, beta, tid, nthr);
                }
                sync_bar();
                for (int rd = 0; rd < NC; ++rd) {
                    const int k2 = rd * NG + gg;
                    g_cols<T, VPT>(a, c, twl, k2, k2 < a.H, tid, nthr);
                }
                sync_bar();
                for (int rd = 0; rd < NR; ++rd) {
                    const int pr = rd * NG + gg;
                    g_rows_inv<T, VPT>(a, c, twl, pr, pr < NP, dg, cc, tid, nthr, pq);
                }
            } else {
                // d = 1: one group does the p update, FFT, symbol, inverse FFT, q
                const bool act = gg == 0;
                T pv[VPT], zv[VPT], pold[VPT], sy[VPT], dv[VPT];
#pragma unroll
                for (int u = 0; u < VPT; ++u) {
                    const int j = tid + u * nthr;
                    zv[u] = pold[u] = dv[u] = T(0);
                    sy[u] = a.sym[j];
                    if (act && j < N) {
                        zv[u] = a.zz[j];
                        if (beta != T(0)) pold[u] = a.p[j];
                        if (dg) dv[u] = dg[j];
                    }
                }
#pragma unroll
                for (int u = 0; u < VPT; ++u) {
                    const int j = tid + u * nthr;
                    pv[u] = zv[u] + beta * pold[u];
                    if (act && j < N) a.p[j] = pv[u];
                    c[lx(j)] = {pv[u], T(0)};
                }
                __syncthreads();
                fft_lds<T, VPT, false, true>(c, a.L, twl, tid, nthr);
#pragma unroll
                for (int u = 0; u < VPT; ++u) {
                    const int k = tid + u * nthr;
                    c[lx(k)] = {c[lx(k)].x * sy[u], c[lx(k)].y * sy[u]};
                }
                __syncthreads();
                fft_lds<T, VPT, true, true>(c, a.L, twl, tid, nthr);
                if (act) {
#pragma unroll
                    for (int u = 0; u < VPT; ++u) {
                        const int j = tid + u * nthr;
                        if (j < N) {
                            const T qv = dv[u] * pv[u] + cc * c[lx(j)].x;
                            a.q[j] = qv;
                            pq += pv[u] * qv;
                        }
                    }
                }
                __syncthreads();
            }
            {
                const int sl[1] = {SL_PQ};
                const T vv[1] = {pq};
                phase_sync<1, true, -1>(a.part, a.bar, a.bar_ticks, sl, vv, red, tot, ph, a.vb, a.vg);
            }
            const double pqt = tot[SL_PQ];
            const T alpha = T(pqt != 0.0 ? rz / pqt : 0.0);
            // x += alpha p, r -= alpha q, (r, r), and pass A of z = M^{-1} r
            prec_A(true, alpha);
            ++it;
            rrt = tot[SL_RR];
            if (rrt <= a.tol2 * bbt || it >= a.maxit || !(rrt == rrt)) break;
            const double rz_new = tot[SL_RZ];
            beta = T(rz != 0.0 ? rz_new / rz : 0.0);
            rz = rz_new;
        }
        total_it += it;
        }
    }
    // the segment's last step: y_{sb-1} = x (grid-stride ownership: in the tau-block mode x was
    // last written by row-owning groups, so the grid synchronises first)
    if constexpr (TB) sync_bar();
    for (long long j = gtid; j < Nd; j += gthreads) a.y[(long long)(sb - 1) * Nd + j] = a.x[j];
    if (a.vb == 0 && threadIdx.x == 0) *a.iters += total_it;
}


// One problem per launch: the grid is the problem's.
template <typename T, int VPT, int MODE, int LC, bool TB>
__global__ __launch_bounds__(kSegBlock) void pinv_segment(PinvArgs<T> a, int sa, int sb) {
    a.vb = blockIdx.x;
    a.vg = gridDim.x;
    segment_run<T, VPT, MODE, LC, TB>(a, sa, sb);
}

// Several problems in one launch (their P^-1 take the same kernel form): problem i owns the workgroups
// [off[i], off[i+1]) and runs the steps [range[i].x, range[i].y) of its forward substitution with its
// own arguments, work buffers and barrier; a problem with no steps in this launch has no workgroups.
template <typename T, int VPT, int MODE>
__global__ __launch_bounds__(kSegBlock) void pinv_segment_multi(const PinvArgs<T>* __restrict__ args,
                                                                const int* __restrict__ off,
                                                                const int2* __restrict__ range, int nprob) {
    int i = 0;
    while (i + 1 < nprob && (int)blockIdx.x >= off[i + 1]) ++i;
    PinvArgs<T> a = args[i];
    a.vb = (int)blockIdx.x - off[i];
    a.vg = off[i + 1] - off[i];
    segment_run<T, VPT, MODE, 0, false>(a, range[i].x, range[i].y);
}

// ---------------------------------------------------------------------------
// host side: work buffers and the segment launches
// ---------------------------------------------------------------------------
template <typename T>
struct PersistentWork {
    T* buf = nullptr;       // x r zz p q rhs bxb bxb2: 8 Nd, then hacc: kHB Nd
    T* tt = nullptr;        // t1, t2: N ns each (2D)
    cplx<T>* spec = nullptr;  // [H][ns] (2D)
    double* part = nullptr;   // kRing * kMaxGrid * kNPart reduction slots
    unsigned* bar = nullptr;  // [1] abort word
    long long* iters = nullptr;
    ResidencyTicket ticket;   // CU slots of the grid while its segments run
};


template <typename T>
void ensure_work(Problem& P, PersistentWork<T>& W);

// The kernel arguments of one problem's forward substitution on the work buffers W.
template <typename T>
PinvArgs<T> make_pinv_args(Problem& P, const Dev<T>& D, PersistentWork<T>& W, const T* z, T* y, double inner_tol,
                           int inner_maxit, int extrap) {
    PinvArgs<T> a{};
    a.d = P.d;
    a.N = P.N;
    a.M = P.M;
    a.L = P.L;
    a.H = P.H;
    a.Nd = P.Nd;
    a.use_tau = (P.tau_ok || P.tau_pad) ? 1 : 0;
    a.Nt = P.Nt;
    a.extrap = extrap;
    a.z = z;
    a.y = y;
    a.g1 = D.gamma1;
    a.g2 = D.gamma2;
    a.dg = D.dg;
    a.epad = D.epad;
    a.sym = D.sym;
    a.tau = D.tau;
    a.tw = D.tw;
    a.sigma = P.sweep_sigma ? P.sweep_sigma : P.d_sigma;
    a.adj = P.adjoint_sweep ? 1 : 0;
    a.ct = T(P.ct);
    a.cf = T(P.cf);
    a.a0 = T(P.a0);
    a.tol2 = inner_tol * inner_tol;
    a.maxit = inner_maxit;
    T* b = W.buf;
    const long long Nd = P.Nd;
    a.x = b;
    a.r = b + Nd;
    a.zz = b + 2 * Nd;
    a.p = b + 3 * Nd;
    a.q = b + 4 * Nd;
    a.rhs = b + 5 * Nd;
    a.bxb = b + 6 * Nd;
    a.bxb2 = b + 7 * Nd;
    a.hacc = b + 8 * Nd;
    a.ns = spec_stride(P.N);
    a.nt = spec_stride(P.Nt);
    a.t1 = W.tt;                                                   // [Nt][nt]
    a.t2 = W.tt ? W.tt + (long long)P.Nt * a.nt : nullptr;  // [N][nt]
    a.spec = W.spec;
    a.part = W.part;
    a.bar = W.bar;
    a.iters = W.iters;
    return a;
}

template <typename T, int VPT, int MODE, int LC, bool TB>
void launch_segments(Problem& P, const Dev<T>& D, PersistentWork<T>& W, const T* z, T* y, double inner_tol,
                     int inner_maxit, bool last_block, int extrap, int blocks, hipStream_t st) {
    PinvArgs<T> a = make_pinv_args<T>(P, D, W, z, y, inner_tol, inner_maxit, extrap);
    const long long Nd = P.Nd;
    const int nthr = P.L / VPT;
    int dev = 0, ncu = 0;
    TSFDE_HIP(hipGetDevice(&dev));
    TSFDE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // The segment kernel's workgroups wait for each other, so all of them must be resident at once,
    // also beside the persistent grids of other streams: the grid is sized to its share of the
    // device's CU slots and holds them (W.ticket) until the host has seen the last segment finish
    // (residency.hpp).  Inside a batch, where up to kMaxInflight problems run side by side, a grid is
    // further limited to ncu / kMaxInflight workgroups, so that that many fit together.
    ResidencyBudget& pool = residency_budget(dev, ncu);
    struct Cfg {
        int block, gpb, grid;
        size_t lds;
    };
    // a workgroup of `block` threads; ring: with the near-history ring in LDS
    auto configure = [&](int block, bool ring) -> Cfg {
        Cfg c{block, block / nthr, 1, 0};
        c.lds = sizeof(cplx<T>) * ((tw_in_lds<T>(VPT) ? P.L : 0) + (size_t)c.gpb * lds_len(P.L)) +
                (ring ? sizeof(T) * (size_t)kNear * (VPT / 2) * 2 * block : 0);
        if (c.lds > 160 * 1024) return Cfg{0, 0, 0, 0};
        // 2D: enough groups that the L/2+1 spectral rows take two rounds
        if (P.d == 2) {
            c.grid = (P.H + 2 * c.gpb - 1) / (2 * c.gpb);
            if (blocks > 0) c.grid = blocks;
        }
        int per_cu = 0;
        TSFDE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pinv_segment<T, VPT, MODE, LC, TB>, block, c.lds));
        if (per_cu < 1) return Cfg{0, 0, 0, 0};
        int cap = std::min(per_cu * ncu, residency_max_grid(pool.total(), kXcds));
        if (shared_launch()) cap = std::min(cap, std::max(1, ncu / kMaxInflight));
        c.grid = std::max(1, std::min({c.grid, cap, kMaxGrid}));
        return c;
    };
    // 2D sine-transform path: workgroups of two (else one) transform groups with the segment's earlier
    // solutions of their own points in LDS, when that fits and the grid takes the row pairs in one
    // round (each thread then owns the same points in every step of the segment)
    Cfg cfg{0, 0, 0, 0};
    a.ring = 0;
    const char* ring_env = std::getenv("TSFDE_PINV_RING");  // diagnostics: 0 keeps the ring off
    if (MODE == SEG_2D_TAU && blocks <= 0 && !(ring_env && std::atoi(ring_env) == 0)) {
        for (int g2 = 2; g2 >= 1 && a.ring == 0; --g2) {
            if (g2 * nthr > kSegBlock || g2 * nthr < kWave) continue;  // phase_sync polls with one full wave
            const Cfg c = configure(g2 * nthr, true);
            if (c.block > 0 && (long long)c.grid * c.gpb >= (P.N + 1) / 2) {
                cfg = c;
                a.ring = 1;
            }
        }
    }
    if (!a.ring) cfg = configure(P.d == 2 ? kSegBlock : nthr, false);
    if (cfg.block == 0) throw HipError{hipErrorInvalidConfiguration, "persistent P^-1: a workgroup does not fit a CU"};
    const int block = cfg.block, grid = cfg.grid;
    const size_t lds = cfg.lds;
    a.bar_ticks = barrier_ticks(dev);
    if (P.capturing) {
        // inside a captured graph: the solver holds the slots around each replay and zeroes the
        // counter before it (the count then adds up over the cycle)
        P.graph_slots = std::max(P.graph_slots, residency_slots(grid, kXcds));
    } else {
        W.ticket.hold(&pool, residency_slots(grid, kXcds));
        launch_fill(reinterpret_cast<float*>(W.iters), 2, 0.0f, st);  // zero the iteration counter
    }
    const int s_last = last_block ? P.M : P.M - 1;
    for (int sa = 0; sa <= s_last; sa += kHB) {
        int sa_ = sa;
        int sb_ = std::min(sa + kHB, s_last + 1);
        const int cnt = std::min(kHB, P.M - sa);
        if (cnt > 0) {
            if (P.adjoint_sweep)  // transposed sweep: unscaled right-hand sides, weights per earlier step
                hipLaunchKernelGGL(far_history<T>, dim3((unsigned)((Nd + 63) / 64)), dim3(256), 0, st, y, a.hacc,
                                   D.epad, z, (const T*)nullptr, (const T*)nullptr, sa, cnt, Nd, D.dg);
            else
                hipLaunchKernelGGL(far_history<T>, dim3((unsigned)((Nd + 63) / 64)), dim3(256), 0, st, y, a.hacc,
                                   D.epad, z, D.gamma1, D.gamma2, sa, cnt, Nd, (const T*)nullptr);
            TSFDE_HIP(hipGetLastError());
        }
        launch_fill(reinterpret_cast<unsigned long long*>(W.part), (long long)kMaxGrid * kNPart, kEmpty, st);  // ring 0
        void* args[] = {&a, &sa_, &sb_};
        TSFDE_HIP(hipLaunchKernel((void*)pinv_segment<T, VPT, MODE, LC, TB>, dim3(grid), dim3(block), args, lds, st));
    }
}

// ---------------------------------------------------------------------------
// Several problems' forward substitutions in shared launches (pinv_segment_multi): all of them take the
// same kernel form (VPT, MODE, run-time length, CG blocks) and, in 1D, the same transform length.
// Problem i keeps the grid it would have alone (2D: two rounds over the spectral rows; 1D: one
// workgroup); a launch takes as many problems as fit the device's CU slots together (chunks), and
// runs one block of kHB steps of each (a round); far_history runs per problem between rounds.  The
// launch tables of every chunk and round are built on the host and copied to the device once.
// ---------------------------------------------------------------------------
template <typename T>
struct MultiItem {
    Problem* P;
    PersistentWork<T>* W;
    PinvArgs<T> a;
    int grid;
    int s_last;
};

template <typename T, int VPT, int MODE>
void launch_segments_multi(std::vector<MultiItem<T>>& items, hipStream_t st) {
    const int n = (int)items.size();
    if (n == 0) return;
    const int L0 = items[0].P->L;
    const int nthr0 = L0 / VPT;
    const int block = (MODE != SEG_1D) ? kSegBlock : nthr0;
    size_t lds = 0;
    for (auto& it : items) {
        if (MODE == SEG_1D && it.P->L != L0) throw HipError{hipErrorInvalidValue, "multi P^-1: 1D problems of one launch share L"};
        const int nthr = it.P->L / VPT;
        const int gpb = block / nthr;
        const size_t l = sizeof(cplx<T>) * ((tw_in_lds<T>(VPT) ? it.P->L : 0) + (size_t)gpb * lds_len(it.P->L));
        lds = std::max(lds, l);
        it.grid = (MODE != SEG_1D) ? std::max(1, (it.P->H + 2 * gpb - 1) / (2 * gpb)) : 1;
        it.s_last = it.P->M;  // the last block row included
    }
    if (lds > 160 * 1024) throw HipError{hipErrorInvalidConfiguration, "multi P^-1 LDS size"};
    int per_cu = 0, dev = 0, ncu = 0;
    TSFDE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pinv_segment_multi<T, VPT, MODE>, block, lds));
    TSFDE_HIP(hipGetDevice(&dev));
    TSFDE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (per_cu < 1) throw HipError{hipErrorInvalidConfiguration, "multi P^-1: a workgroup does not fit a CU"};
    ResidencyBudget& pool = residency_budget(dev, ncu);
    const int cap = std::min({per_cu * ncu, residency_max_grid(pool.total(), kXcds), kMaxGrid});
    const unsigned long long ticks = barrier_ticks(dev);
    for (auto& it : items) {
        it.grid = std::min(it.grid, cap);
        it.a.bar_ticks = ticks;
    }
    // chunks of problems whose grids fit together
    std::vector<int> cstart{0};
    for (int i = 0, g = 0; i < n; ++i) {
        if (g > 0 && g + items[i].grid > cap) {
            cstart.push_back(i);
            g = 0;
        }
        g += items[i].grid;
    }
    cstart.push_back(n);
    const int nchunk = (int)cstart.size() - 1;
    int rounds = 0;
    for (auto& it : items) rounds = std::max(rounds, (it.s_last + kHB) / kHB);
    // launch tables: per chunk and round, [args x k][off x (k + 1)][range x k], 16-byte aligned
    auto al = [](size_t v) { return (v + 15) & ~size_t(15); };
    struct Launch {
        size_t o_args, o_off, o_range;
        int k, grid, chunk, round;
    };
    std::vector<Launch> launches;
    size_t bytes = 0;
    for (int c = 0; c < nchunk; ++c)
        for (int r = 0; r < rounds; ++r) {
            int k = 0, g = 0;
            for (int i = cstart[c]; i < cstart[c + 1]; ++i)
                if (r * kHB <= items[i].s_last) {
                    ++k;
                    g += items[i].grid;
                }
            if (k == 0) continue;
            Launch l{};
            l.k = k;
            l.grid = g;
            l.chunk = c;
            l.round = r;
            l.o_args = bytes;
            bytes = al(bytes + sizeof(PinvArgs<T>) * k);
            l.o_off = bytes;
            bytes = al(bytes + sizeof(int) * (k + 1));
            l.o_range = bytes;
            bytes = al(bytes + sizeof(int2) * k);
            launches.push_back(l);
        }
    Problem& P0 = *items[0].P;
    if (P0.multi_bytes < bytes) {
        if (P0.multi_dev) (void)hipFree(P0.multi_dev);
        if (P0.multi_host) (void)hipHostFree(P0.multi_host);
        P0.multi_dev = nullptr;
        P0.multi_host = nullptr;
        P0.multi_bytes = 0;
        TSFDE_HIP(hipMalloc(&P0.multi_dev, bytes));
        TSFDE_HIP(hipHostMalloc(&P0.multi_host, bytes, hipHostMallocDefault));
        P0.multi_bytes = bytes;
    }
    unsigned char* hb = static_cast<unsigned char*>(P0.multi_host);
    for (const Launch& l : launches) {
        auto* args = reinterpret_cast<PinvArgs<T>*>(hb + l.o_args);
        int* off = reinterpret_cast<int*>(hb + l.o_off);
        int2* range = reinterpret_cast<int2*>(hb + l.o_range);
        int k = 0, g = 0;
        for (int i = cstart[l.chunk]; i < cstart[l.chunk + 1]; ++i) {
            const int sa = l.round * kHB;
            if (sa > items[i].s_last) continue;
            args[k] = items[i].a;
            off[k] = g;
            range[k] = make_int2(sa, std::min(sa + kHB, items[i].s_last + 1));
            g += items[i].grid;
            ++k;
        }
        off[k] = g;
    }
    TSFDE_HIP(hipMemcpyAsync(P0.multi_dev, P0.multi_host, bytes, hipMemcpyHostToDevice, st));
    int gmax = 0;
    for (const Launch& l : launches) gmax = std::max(gmax, l.grid);
    ResidencyTicket ticket;
    struct Release {
        ResidencyTicket& t;
        ~Release() { t.release(); }
    } release{ticket};
    ticket.hold(&pool, residency_slots(gmax, kXcds));
    for (auto& it : items) {
        launch_fill(reinterpret_cast<float*>(it.W->iters), 2, 0.0f, st);
        launch_fill(reinterpret_cast<float*>(it.W->bar) + 1, 1, 0.0f, st);  // abort word
    }
    unsigned char* db = static_cast<unsigned char*>(P0.multi_dev);
    for (const Launch& l : launches) {
        const int sa = l.round * kHB;
        for (int i = cstart[l.chunk]; i < cstart[l.chunk + 1]; ++i) {
            MultiItem<T>& it = items[i];
            if (sa > it.s_last) continue;
            Problem& P = *it.P;
            const int cnt = std::min(kHB, P.M - sa);
            if (cnt > 0) {
                hipLaunchKernelGGL(far_history<T>, dim3((unsigned)((P.Nd + 63) / 64)), dim3(256), 0, st, it.a.y,
                                   it.a.hacc, it.a.epad, it.a.z, it.a.g1, it.a.g2, sa, cnt, P.Nd, (const T*)nullptr);
                TSFDE_HIP(hipGetLastError());
            }
            launch_fill(reinterpret_cast<unsigned long long*>(it.W->part), (long long)kMaxGrid * kNPart, kEmpty,
                        st);  // ring 0 of the reduction slots
        }
        hipLaunchKernelGGL((pinv_segment_multi<T, VPT, MODE>), dim3(l.grid), dim3(block), lds, st,
                           reinterpret_cast<const PinvArgs<T>*>(db + l.o_args), reinterpret_cast<const int*>(db + l.o_off),
                           reinterpret_cast<const int2*>(db + l.o_range), l.k);
        TSFDE_HIP(hipGetLastError());
    }
    // iteration counts and abort words, then the host sees the last round finish
    for (int i = 0; i < n; ++i) {
        long long* ith = reinterpret_cast<long long*>(items[i].P->host_scalars + 56);
        unsigned* abh = reinterpret_cast<unsigned*>(items[i].P->host_scalars + 57);
        TSFDE_HIP(hipMemcpyAsync(ith, items[i].W->iters, sizeof(long long), hipMemcpyDeviceToHost, st));
        TSFDE_HIP(hipMemcpyAsync(abh, items[i].W->bar + 1, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    }
    TSFDE_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i)
        if (*reinterpret_cast<unsigned*>(items[i].P->host_scalars + 57) != 0u)
            throw HipError{hipErrorLaunchTimeOut, "multi P^-1: a device-wide barrier wait timed out"};
}

// launches of the fixed-length 2D sine-transform kernels (CG blocks: pinv_fixed.hip; tau blocks:
// pinv_fixed_tau.hip); false if L has no fixed-length kernel
template <typename T>
bool launch_segments_fixed(Problem& P, const Dev<T>& D, PersistentWork<T>& W, const T* z, T* y, double inner_tol,
                           int inner_maxit, bool last_block, int extrap, int blocks, hipStream_t st);
template <typename T>
bool launch_segments_fixed_tau(Problem& P, const Dev<T>& D, PersistentWork<T>& W, const T* z, T* y, bool last_block,
                               int blocks, hipStream_t st);

}  // namespace tsfde
