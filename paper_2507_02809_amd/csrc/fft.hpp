// LDS-resident Stockham FFT for power-of-two lengths (radix 8, with one radix-4 or
// radix-2 pass when log2(L) is not a multiple of 3).
//
// A group of `nthr` threads transforms one sequence of L = VPT * nthr complex values
// held in LDS; several groups of a workgroup may run side by side on their own
// sequences (every group executes the same passes, so the passes synchronise with
// __syncthreads()).  Each pass reads all its butterfly inputs into registers, waits,
// and writes the outputs in Stockham (self-sorting) order in place.
//
// Twiddles come from a table tw[m] = exp(-2 pi i m / L), m = 0..L-1, computed on
// the host in double precision (rounded once for FP32).  Forward transforms use
// exp(-2 pi i jk/L); the inverse uses the conjugate and is not scaled.
#pragma once

#include "common.hpp"

namespace tsfde {

// LDS sequences are stored with one pad slot after every 8 complex values: the Stockham write
// a[(b - k) R + k + r Ns] otherwise sends all 64 lanes of a wave to the same LDS banks (a stride of
// 8 complex values is 128 bytes); with the pad each 128-bit access is spread over all banks.
__host__ __device__ __forceinline__ constexpr int lx(int i) { return i + (i >> 3); }
__host__ __device__ __forceinline__ constexpr int lds_len(int L) { return L + (L >> 3); }

template <typename T, bool INV>
__device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) {  // * (-i) forward, * (+i) inverse
    return INV ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cplx<T>& x0, cplx<T>& x1, cplx<T>& x2, cplx<T>& x3) {
    cplx<T> a = cadd(x0, x2), b = csub(x0, x2);
    cplx<T> c = cadd(x1, x3), d = mul_mi<T, INV>(csub(x1, x3));
    x0 = cadd(a, c);
    x2 = csub(a, c);
    x1 = cadd(b, d);
    x3 = csub(b, d);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cplx<T>* v) {
    // even / odd halves, then combine with W8^k
    cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<T, INV>(e0, e1, e2, e3);
    dft4<T, INV>(o0, o1, o2, o3);
    const T r = T(0.70710678118654752440084436210484903928);
    // W8^1 = (1 - i)/sqrt2 forward, (1 + i)/sqrt2 inverse
    cplx<T> t1 = INV ? cplx<T>{r * (o1.x - o1.y), r * (o1.x + o1.y)}
                     : cplx<T>{r * (o1.x + o1.y), r * (o1.y - o1.x)};
    cplx<T> t2 = mul_mi<T, INV>(o2);
    // W8^3 = (-1 - i)/sqrt2 forward, (-1 + i)/sqrt2 inverse
    cplx<T> t3 = INV ? cplx<T>{-r * (o3.x + o3.y), r * (o3.x - o3.y)}
                     : cplx<T>{r * (o3.y - o3.x), -r * (o3.x + o3.y)};
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, t1);
    v[5] = csub(e1, t1);
    v[2] = cadd(e2, t2);
    v[6] = csub(e2, t2);
    v[3] = cadd(e3, t3);
    v[7] = csub(e3, t3);
}

template <typename T, int R, int VPT, bool INV, bool HT>
__device__ __forceinline__ void stockham_pass(cplx<T>* a, int L, int Ns, const cplx<T>* __restrict__ tw,
                                              int tid, int nthr) {
    constexpr int NB = VPT / R;  // butterflies per thread
    // HT with one butterfly per thread: its twiddles are read together with the data, before the
    // barrier (they do not depend on it).  It pays where a pass waits on LDS latency (the persistent
    // P^-1 kernels); the streaming matvec kernels, which hide that latency with other workgroups,
    // ran slower with it (the registers it holds), so they leave HT off
    constexpr bool HOIST = HT && NB == 1;
    const int nbut = L / R;
    const int tstride = L / (Ns * R);
    cplx<T> v[NB][R], w[HOIST ? R : 1];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int b = tid + c * nthr;
#pragma unroll
        for (int r = 0; r < R; ++r) v[c][r] = a[lx(b + r * nbut)];
    }
    if (HOIST && Ns > 1) {
        const int k = tid & (Ns - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) w[HOIST ? r : 0] = tw[r * k * tstride];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int b = tid + c * nthr;
        const int k = b & (Ns - 1);
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cplx<T> t = HOIST ? w[HOIST ? r : 0] : tw[r * k * tstride];
                v[c][r] = INV ? cmulc(v[c][r], t) : cmul(v[c][r], t);
            }
        }
        if constexpr (R == 8) {
            dft8<T, INV>(v[c]);
        } else if constexpr (R == 4) {
            dft4<T, INV>(v[c][0], v[c][1], v[c][2], v[c][3]);
        } else {
            dft2<T, INV>(v[c]);
        }
        const int base = (b - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) a[lx(base + r * Ns)] = v[c][r];
    }
    __syncthreads();
}

// In-place FFT of a[0..L) (stored with the lx() padding) with L = VPT * nthr.  Must be called by all threads of the
// workgroup (it contains __syncthreads()); `tid` is the thread's index within its group.
template <typename T, int VPT, bool INV, bool HT = false>
__device__ __forceinline__ void fft_lds(cplx<T>* a, int L, const cplx<T>* __restrict__ tw, int tid, int nthr) {
    int Ns = 1;
    while (Ns < L) {
        const int rem = L / Ns;
        if (rem >= 8) {
            stockham_pass<T, 8, VPT, INV, HT>(a, L, Ns, tw, tid, nthr);
            Ns *= 8;
        } else if (rem == 4) {
            stockham_pass<T, 4, VPT, INV, HT>(a, L, Ns, tw, tid, nthr);
            Ns *= 4;
        } else {
            stockham_pass<T, 2, VPT, INV, HT>(a, L, Ns, tw, tid, nthr);
            Ns *= 2;
        }
    }
}

// ---------------------------------------------------------------------------
// Register-resident variant.  Thread tid of a group holds v[u] = a_{tid + u nthr}, u < VPT (the
// "natural" layout).  The first Stockham pass reads exactly those positions and the last pass writes
// exactly those positions, so with IN_REG the input is taken from v (no LDS write and barrier before
// the first pass) and with OUT_REG the output is left in v (no LDS read after the last pass); LDS
// carries only the exchanges between passes.
//   IN_REG:  on entry the LDS sequence must be free to overwrite (no thread still reading it);
//   !IN_REG: the input is in LDS and visible to the group;
//   OUT_REG: on exit the LDS sequence holds scratch data and may be overwritten at once;
//   !OUT_REG: on exit the output is in LDS and visible to the group.
// ---------------------------------------------------------------------------
template <typename T, int R, int VPT, bool INV, bool HT>
__device__ __forceinline__ void stockham_pass_x(cplx<T> (&v)[VPT], cplx<T>* a, int L, int Ns,
                                                const cplx<T>* __restrict__ tw, int tid, int nthr, bool in_reg,
                                                bool out_reg) {
    constexpr int NB = VPT / R;  // butterflies per thread
    constexpr bool HOIST = HT && NB == 1;  // twiddles read before the data wait (as in stockham_pass)
    const int nbut = L / R;
    const int tstride = L / (Ns * R);
    cplx<T> w[NB][R], tt[HOIST ? R : 1];
    if (HOIST && Ns > 1) {
        const int k = tid & (Ns - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) tt[HOIST ? r : 0] = tw[r * k * tstride];
    }
    if (in_reg) {
        // butterfly (b = tid + c nthr, r) reads position b + r L/R = tid + (c + NB r) nthr
#pragma unroll
        for (int c = 0; c < NB; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) w[c][r] = v[c + NB * r];
    } else {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int b = tid + c * nthr;
#pragma unroll
            for (int r = 0; r < R; ++r) w[c][r] = a[lx(b + r * nbut)];
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int b = tid + c * nthr;
        const int k = b & (Ns - 1);
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cplx<T> t = HOIST ? tt[HOIST ? r : 0] : tw[r * k * tstride];
                w[c][r] = INV ? cmulc(w[c][r], t) : cmul(w[c][r], t);
            }
        }
        if constexpr (R == 8) {
            dft8<T, INV>(w[c]);
        } else if constexpr (R == 4) {
            dft4<T, INV>(w[c][0], w[c][1], w[c][2], w[c][3]);
        } else {
            dft2<T, INV>(w[c]);
        }
    }
    if (out_reg) {
        // last pass (Ns = L/R): butterfly (b, r) writes position b + r Ns = tid + (c + NB r) nthr
#pragma unroll
        for (int c = 0; c < NB; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) v[c + NB * r] = w[c][r];
    } else {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int b = tid + c * nthr;
            const int k = b & (Ns - 1);
            const int base = (b - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) a[lx(base + r * Ns)] = w[c][r];
        }
        __syncthreads();
    }
}

template <typename T, int VPT, bool INV, bool IN_REG, bool OUT_REG, bool HT = false>
__device__ __forceinline__ void fft_x(cplx<T> (&v)[VPT], cplx<T>* a, int L, const cplx<T>* __restrict__ tw, int tid,
                                      int nthr) {
    int Ns = 1;
    while (Ns < L) {
        const int rem = L / Ns;
        const bool first = (Ns == 1);
        const int R = rem >= 8 ? 8 : rem;
        const bool last = (Ns * R == L);
        const bool in_reg = IN_REG && first;
        const bool out_reg = OUT_REG && last;
        if (R == 8) {
            stockham_pass_x<T, 8, VPT, INV, HT>(v, a, L, Ns, tw, tid, nthr, in_reg, out_reg);
        } else if (R == 4) {
            stockham_pass_x<T, 4, VPT, INV, HT>(v, a, L, Ns, tw, tid, nthr, in_reg, out_reg);
        } else {
            stockham_pass_x<T, 2, VPT, INV, HT>(v, a, L, Ns, tw, tid, nthr, in_reg, out_reg);
        }
        Ns *= R;
    }
}

}  // namespace tsfde
