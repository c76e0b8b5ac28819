// Spectral kernels: the Toeplitz product B y through a zero-padded circulant embedding
// (§5 matvec step 1(b): embed B_n in a d-level circulant, FFT, multiply by the circulant's
// eigenvalues, inverse FFT, crop) and the tau preconditioner S diag(.) S of B through the
// sine transform (§5 Remark), both built on the LDS Stockham FFT of fft.hpp.
//
// One workgroup transforms one sequence of length L (blockDim = L / VPT threads).
//
// d = 2 Toeplitz product, slices of N x N reals (row i, column j, j fastest):
//   rows_fwd : pairs of rows (i, i+1) packed as real + i*imag, zero-padded to L, FFT over j;
//              the two half spectra (k2 = 0..L/2) are separated and stored transposed in
//              spec[slice][k2][i]  (complex, H = L/2+1 rows of N).
//   cols     : each spec row k2 (N complex values over i) zero-padded to L, FFT over i,
//              times sym[k2][k1] = lambda(k1,k2)/L^2, inverse FFT, first N values kept.
//   rows_inv : the two half spectra of rows (i, i+1) are re-packed into one Hermitian-
//              completed spectrum, inverse FFT over k2, real/imag parts are rows i / i+1;
//              an epilogue writes the operator output.
// d = 1: one kernel per pair of vectors: pack, FFT, multiply, inverse FFT, epilogue.
#include "fft.hpp"
#include "internal.hpp"

namespace tsfde {

enum Epi : int { EPI_MATVEC = 0, EPI_SPD = 1 };

template <typename T>
struct EpiArgs {
    // EPI_MATVEC: slice s < M: z[s] += ct * gamma2[s] .* u;  s == M: z[M] = cf * gamma2[M-1] .* u + ylast
    // (ylast = y[M-1] for A; gamma2 null stands for ones)
    T* z;
    const T* ylast;
    const T* gamma2;
    T ct, cf;
    int M;
    // EPI_SPD: q = dg .* p + c * u, partials of (p, q)
    const T* p;
    T* q;
    const T* dg;
    T c;
    T* partials;
};

template <typename T>
__device__ __forceinline__ T epi_apply(const EpiArgs<T>& a, int mode, int slice, long long Nd, long long idx,
                                       T u, T& dotacc) {
    if (mode == EPI_MATVEC) {
        if (slice < a.M) {
            const long long o = (long long)slice * Nd + idx;
            a.z[o] = a.z[o] + a.ct * (a.gamma2 ? a.gamma2[o] : T(1)) * u;
        } else {
            const long long o = (long long)a.M * Nd + idx;
            const long long g = (long long)(a.M - 1) * Nd + idx;
            a.z[o] = a.cf * (a.gamma2 ? a.gamma2[g] : T(1)) * u + a.ylast[idx];
        }
        return T(0);
    } else {
        const T pv = a.p[idx];
        const T qv = (a.dg ? a.dg[idx] * pv : T(0)) + a.c * u;
        a.q[idx] = qv;
        dotacc += pv * qv;
        return qv;
    }
}

// ---------------------------------------------------------------------------
// d = 2 Toeplitz product
// ---------------------------------------------------------------------------

template <typename T, int VPT>
__global__ void toep2d_rows_fwd(const T* __restrict__ x, long long slice_stride, int N, int L,
                                const cplx<T>* __restrict__ tw, cplx<T>* __restrict__ spec) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* c = reinterpret_cast<cplx<T>*>(smem_raw);
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int i0 = 2 * blockIdx.x, i1 = i0 + 1;
    const int slice = blockIdx.y;
    const T* xs = x + slice_stride * slice;
    for (int j = tid; j < L; j += nthr) {
        cplx<T> v = {T(0), T(0)};
        if (j < N) {
            v.x = xs[(long long)i0 * N + j];
            if (i1 < N) v.y = xs[(long long)i1 * N + j];
        }
        c[lx(j)] = v;
    }
    __syncthreads();
    fft_lds<T, VPT, false>(c, L, tw, tid, nthr);
    const int H = L / 2 + 1;
    cplx<T>* out = spec + (long long)slice * H * N;
    for (int k = tid; k < H; k += nthr) {
        const cplx<T> C = c[lx(k)];
        const cplx<T> Cm = c[lx((L - k) & (L - 1))];
        const cplx<T> X0 = {T(0.5) * (C.x + Cm.x), T(0.5) * (C.y - Cm.y)};
        const cplx<T> X1 = {T(0.5) * (C.y + Cm.y), T(0.5) * (Cm.x - C.x)};
        out[(long long)k * N + i0] = X0;
        if (i1 < N) out[(long long)k * N + i1] = X1;
    }
}

template <typename T, int VPT>
__global__ void toep2d_cols(cplx<T>* __restrict__ spec, int N, int L, const cplx<T>* __restrict__ tw,
                            const T* __restrict__ sym) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* c = reinterpret_cast<cplx<T>*>(smem_raw);
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int k2 = blockIdx.x;
    const int H = L / 2 + 1;
    cplx<T>* row = spec + ((long long)blockIdx.y * H + k2) * N;
    for (int i = tid; i < L; i += nthr) c[lx(i)] = (i < N) ? row[i] : cplx<T>{T(0), T(0)};
    __syncthreads();
    fft_lds<T, VPT, false>(c, L, tw, tid, nthr);
    const T* sy = sym + (long long)k2 * L;
    for (int k1 = tid; k1 < L; k1 += nthr) {
        const T s = sy[k1];
        c[lx(k1)] = {c[lx(k1)].x * s, c[lx(k1)].y * s};
    }
    __syncthreads();
    fft_lds<T, VPT, true>(c, L, tw, tid, nthr);
    for (int i = tid; i < N; i += nthr) row[i] = c[lx(i)];
}

template <typename T, int VPT>
__global__ void toep2d_rows_inv(const cplx<T>* __restrict__ spec, int N, int L, const cplx<T>* __restrict__ tw,
                                int slice0, EpiArgs<T> ea, int mode) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* c = reinterpret_cast<cplx<T>*>(smem_raw);
    __shared__ T red[4];
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int i0 = 2 * blockIdx.x, i1 = i0 + 1;
    const int H = L / 2 + 1;
    const cplx<T>* sp = spec + (long long)blockIdx.y * H * N;
    for (int k = tid; k < L; k += nthr) {
        const int kk = (k < H) ? k : L - k;
        const cplx<T> Y0 = sp[(long long)kk * N + i0];
        const cplx<T> Y1 = (i1 < N) ? sp[(long long)kk * N + i1] : cplx<T>{T(0), T(0)};
        c[lx(k)] = (k < H) ? cplx<T>{Y0.x - Y1.y, Y0.y + Y1.x} : cplx<T>{Y0.x + Y1.y, Y1.x - Y0.y};
    }
    __syncthreads();
    fft_lds<T, VPT, true>(c, L, tw, tid, nthr);
    const long long Nd = (long long)N * N;
    const int slice = slice0 + blockIdx.y;
    T dot = T(0);
    for (int j = tid; j < N; j += nthr) {
        const cplx<T> v = c[lx(j)];
        epi_apply(ea, mode, slice, Nd, (long long)i0 * N + j, v.x, dot);
        if (i1 < N) epi_apply(ea, mode, slice, Nd, (long long)i1 * N + j, v.y, dot);
    }
    if (mode == EPI_SPD) {
        T s = block_sum(dot, red);
        if (tid == 0) ea.partials[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// d = 1 Toeplitz product: pairs of vectors (slices 2b, 2b+1) in one complex FFT
// ---------------------------------------------------------------------------

template <typename T, int VPT>
__global__ void toep1d(const T* __restrict__ x, int nvec, int N, int L, const cplx<T>* __restrict__ tw,
                       const T* __restrict__ sym, int slice0, EpiArgs<T> ea, int mode) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* c = reinterpret_cast<cplx<T>*>(smem_raw);
    __shared__ T red[4];
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int a = 2 * blockIdx.x, b = a + 1;
    for (int j = tid; j < L; j += nthr) {
        cplx<T> v = {T(0), T(0)};
        if (j < N) {
            v.x = x[(long long)a * N + j];
            if (b < nvec) v.y = x[(long long)b * N + j];
        }
        c[lx(j)] = v;
    }
    __syncthreads();
    fft_lds<T, VPT, false>(c, L, tw, tid, nthr);
    for (int k = tid; k < L; k += nthr) {
        const T s = sym[k];
        c[lx(k)] = {c[lx(k)].x * s, c[lx(k)].y * s};
    }
    __syncthreads();
    fft_lds<T, VPT, true>(c, L, tw, tid, nthr);
    T dot = T(0);
    for (int j = tid; j < N; j += nthr) {
        const cplx<T> v = c[lx(j)];
        epi_apply(ea, mode, slice0 + a, (long long)N, (long long)j, v.x, dot);
        if (b < nvec) epi_apply(ea, mode, slice0 + b, (long long)N, (long long)j, v.y, dot);
    }
    if (mode == EPI_SPD) {
        T s = block_sum(dot, red);
        if (tid == 0) ea.partials[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// tau preconditioner: DST-I through the FFT of the odd extension of length Ld = 2(N+1)
//   x_ext = [0, x_1..x_N, 0, -x_N..-x_1],  FFT_k = -2i sum_n x_n sin(pi n k/(N+1))
// Two real rows u, v packed as u + i v give DST(u) = -Im/2 and DST(v) = Re/2.
// ---------------------------------------------------------------------------

enum DstMode : int { DST_PLAIN = 0, DST_SCALE = 1, DST_FINAL = 2 };

template <typename T, int VPT>
__global__ void dst2d_rows(const T* __restrict__ x, T* __restrict__ out, int N, int Ld,
                           const cplx<T>* __restrict__ tw, int mode, const T* __restrict__ tau, T sigma,
                           T cfac, T scale, const T* __restrict__ rdot, T* __restrict__ partials) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* c = reinterpret_cast<cplx<T>*>(smem_raw);
    __shared__ T red[4];
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int i0 = 2 * blockIdx.x, i1 = i0 + 1;
    for (int n = tid; n < Ld; n += nthr) {
        cplx<T> v = {T(0), T(0)};
        if (n >= 1 && n <= N) {
            v.x = x[(long long)i0 * N + n - 1];
            if (i1 < N) v.y = x[(long long)i1 * N + n - 1];
        } else if (n >= N + 2) {
            const int m = Ld - n - 1;
            v.x = -x[(long long)i0 * N + m];
            if (i1 < N) v.y = -x[(long long)i1 * N + m];
        }
        c[lx(n)] = v;
    }
    __syncthreads();
    fft_lds<T, VPT, false>(c, Ld, tw, tid, nthr);
    T dot = T(0);
    for (int k = tid; k < N; k += nthr) {
        const cplx<T> C = c[lx(k + 1)];
        T d0 = T(-0.5) * C.y, d1 = T(0.5) * C.x;
        const long long o0 = (long long)k * N + i0, o1 = (long long)k * N + i1;
        if (mode == DST_SCALE) {
            d0 *= scale / (sigma + cfac * tau[(long long)i0 * N + k]);
            if (i1 < N) d1 *= scale / (sigma + cfac * tau[(long long)i1 * N + k]);
        }
        out[o0] = d0;
        if (i1 < N) out[o1] = d1;
        if (mode == DST_FINAL) {
            dot += rdot[o0] * d0;
            if (i1 < N) dot += rdot[o1] * d1;
        }
    }
    if (mode == DST_FINAL) {
        T s = block_sum(dot, red);
        if (tid == 0) partials[blockIdx.x] = s;
    }
}

// d = 1: z = (2/(N+1)) DST(diag(1/(sigma + c tau)) DST(r)), one vector per launch.
template <typename T, int VPT>
__global__ void dst1d_prec(const T* __restrict__ r, T* __restrict__ z, int N, int Ld, const cplx<T>* __restrict__ tw,
                           const T* __restrict__ tau, T sigma, T cfac, T scale, T* __restrict__ partials) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* c = reinterpret_cast<cplx<T>*>(smem_raw);
    __shared__ T red[4];
    const int nthr = blockDim.x, tid = threadIdx.x;
    for (int n = tid; n < Ld; n += nthr) {
        T v = T(0);
        if (n >= 1 && n <= N) v = r[n - 1];
        else if (n >= N + 2) v = -r[Ld - n - 1];
        c[lx(n)] = {v, T(0)};
    }
    __syncthreads();
    fft_lds<T, VPT, false>(c, Ld, tw, tid, nthr);
    // hat_k = DST(r)_k * scale/(sigma + c tau_k), k = 1..N, held in registers before the rebuild
    constexpr int MAXK = VPT;
    T hv[MAXK];
#pragma unroll
    for (int q = 0; q < MAXK; ++q) {
        const int k = tid + q * nthr;  // k indexes 0..N-1 (frequency k+1)
        hv[q] = (k < N) ? T(-0.5) * c[lx(k + 1)].y * scale / (sigma + cfac * tau[k]) : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXK; ++q) {
        const int k = tid + q * nthr;
        if (k < N) {
            c[lx(k + 1)] = {hv[q], T(0)};
            c[lx(Ld - k - 1)] = {-hv[q], T(0)};
        }
    }
    if (tid == 0) {
        c[lx(0)] = {T(0), T(0)};
        c[lx(N + 1)] = {T(0), T(0)};
    }
    __syncthreads();
    fft_lds<T, VPT, false>(c, Ld, tw, tid, nthr);
    T dot = T(0);
    for (int k = tid; k < N; k += nthr) {
        const T v = T(-0.5) * c[lx(k + 1)].y;
        z[k] = v;
        dot += r[k] * v;
    }
    T s = block_sum(dot, red);
    if (tid == 0) partials[0] = s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T>
static int pick_vpt(int L) {
    if (L <= 2048) return 8;
    if (L == 4096) return 16;
    return 32;
}

#define TSFDE_VPT_DISPATCH(VPTV, ...)            \
    switch (VPTV) {                              \
        case 8: { constexpr int VPT = 8; __VA_ARGS__; } break;   \
        case 16: { constexpr int VPT = 16; __VA_ARGS__; } break; \
        default: { constexpr int VPT = 32; __VA_ARGS__; } break; \
    }

template <typename T>
void launch_toeplitz_matvec(const Problem& P, const Dev<T>& D, const T* y, T* z, hipStream_t s, const T* ylast) {
    EpiArgs<T> ea{};
    ea.z = z;
    ea.ylast = ylast ? ylast : y + (long long)(P.M - 1) * P.Nd;
    ea.gamma2 = D.gamma2;
    ea.ct = T(P.ct);
    ea.cf = T(P.cf);
    ea.M = P.M;
    const int L = P.L;
    const int vpt = pick_vpt<T>(L);
    const int nthr = L / vpt;
    const size_t lds = sizeof(cplx<T>) * lds_len(L);
    const int nslices = P.M + 1;
    if (P.d == 1) {
        // one transform per workgroup: as many threads as a workgroup takes (up to 1024), so that a long
        // transform (L = 8192 at N = 4095) has 16 waves to hide its LDS and twiddle latencies rather than 4
        const int vpt1 = std::max(8, L / 1024);
        const int nthr1 = L / vpt1;
        const int npairs = (nslices + 1) / 2;
        TSFDE_VPT_DISPATCH(vpt1, hipLaunchKernelGGL((toep1d<T, VPT>), dim3(npairs), dim3(nthr1), lds, s, y, nslices,
                                                    P.N, L, D.tw, D.sym, 0, ea, (int)EPI_MATVEC));
        TSFDE_HIP(hipGetLastError());
        return;
    }
    // d = 2: process the slices in chunks that fit the spectrum buffer
    const int NP = (P.N + 1) / 2;
    const int H = L / 2 + 1;
    for (int s0 = 0; s0 < nslices; s0 += P.nspec) {
        const int ns = std::min(P.nspec, nslices - s0);
        const T* ys = y + (long long)s0 * P.Nd;
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((toep2d_rows_fwd<T, VPT>), dim3(NP, ns), dim3(nthr), lds, s, ys,
                                                   (long long)P.Nd, P.N, L, D.tw, D.spec));
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((toep2d_cols<T, VPT>), dim3(H, ns), dim3(nthr), lds, s, D.spec,
                                                   P.N, L, D.tw, D.sym));
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((toep2d_rows_inv<T, VPT>), dim3(NP, ns), dim3(nthr), lds, s,
                                                   D.spec, P.N, L, D.tw, s0, ea, (int)EPI_MATVEC));
        TSFDE_HIP(hipGetLastError());
    }
}

template <typename T>
void launch_spd_apply(const Problem& P, const Dev<T>& D, const T* p, T* q, const T* dg, T c, T* partials,
                      int* nparts, hipStream_t s) {
    EpiArgs<T> ea{};
    ea.p = p;
    ea.q = q;
    ea.dg = dg;
    ea.c = c;
    ea.partials = partials;
    const int L = P.L;
    const int vpt = pick_vpt<T>(L);
    const int nthr = L / vpt;
    const size_t lds = sizeof(cplx<T>) * lds_len(L);
    if (P.d == 1) {
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((toep1d<T, VPT>), dim3(1), dim3(nthr), lds, s, p, 1, P.N, L,
                                                   D.tw, D.sym, 0, ea, (int)EPI_SPD));
        *nparts = 1;
    } else {
        const int NP = (P.N + 1) / 2;
        const int H = L / 2 + 1;
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((toep2d_rows_fwd<T, VPT>), dim3(NP, 1), dim3(nthr), lds, s, p,
                                                   (long long)P.Nd, P.N, L, D.tw, D.spec));
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((toep2d_cols<T, VPT>), dim3(H, 1), dim3(nthr), lds, s, D.spec,
                                                   P.N, L, D.tw, D.sym));
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((toep2d_rows_inv<T, VPT>), dim3(NP, 1), dim3(nthr), lds, s,
                                                   D.spec, P.N, L, D.tw, 0, ea, (int)EPI_SPD));
        *nparts = NP;
    }
    TSFDE_HIP(hipGetLastError());
}

template <typename T>
void launch_tau_prec(const Problem& P, const Dev<T>& D, const T* r, T* z, T sigma, T c, T* partials, int* nparts,
                     hipStream_t s) {
    const int Ld = P.Ld;
    const int vpt = pick_vpt<T>(Ld);
    const int nthr = Ld / vpt;
    const size_t lds = sizeof(cplx<T>) * lds_len(Ld);
    const T scale1 = T(2.0 / (P.N + 1));
    if (P.d == 1) {
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((dst1d_prec<T, VPT>), dim3(1), dim3(nthr), lds, s, r, z, P.N, Ld,
                                                   D.twd, D.tau, sigma, c, scale1, partials));
        *nparts = 1;
    } else {
        const int NP = (P.N + 1) / 2;
        T* t1 = D.pcg + 5 * P.Nd;
        T* t2 = D.pcg + 6 * P.Nd;
        const T scale = scale1 * scale1;
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((dst2d_rows<T, VPT>), dim3(NP), dim3(nthr), lds, s, r, t1, P.N, Ld,
                                                   D.twd, (int)DST_PLAIN, D.tau, sigma, c, scale, r, partials));
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((dst2d_rows<T, VPT>), dim3(NP), dim3(nthr), lds, s, t1, t2, P.N, Ld,
                                                   D.twd, (int)DST_SCALE, D.tau, sigma, c, scale, r, partials));
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((dst2d_rows<T, VPT>), dim3(NP), dim3(nthr), lds, s, t2, t1, P.N, Ld,
                                                   D.twd, (int)DST_PLAIN, D.tau, sigma, c, scale, r, partials));
        TSFDE_VPT_DISPATCH(vpt, hipLaunchKernelGGL((dst2d_rows<T, VPT>), dim3(NP), dim3(nthr), lds, s, t1, z, P.N, Ld,
                                                   D.twd, (int)DST_FINAL, D.tau, sigma, c, scale, r, partials));
        *nparts = NP;
    }
    TSFDE_HIP(hipGetLastError());
}

template void launch_toeplitz_matvec<double>(const Problem&, const Dev<double>&, const double*, double*, hipStream_t,
                                             const double*);
template void launch_toeplitz_matvec<float>(const Problem&, const Dev<float>&, const float*, float*, hipStream_t,
                                            const float*);
template void launch_spd_apply<double>(const Problem&, const Dev<double>&, const double*, double*, const double*,
                                       double, double*, int*, hipStream_t);
template void launch_spd_apply<float>(const Problem&, const Dev<float>&, const float*, float*, const float*, float,
                                      float*, int*, hipStream_t);
template void launch_tau_prec<double>(const Problem&, const Dev<double>&, const double*, double*, double, double,
                                      double*, int*, hipStream_t);
template void launch_tau_prec<float>(const Problem&, const Dev<float>&, const float*, float*, float, float, float*,
                                     int*, hipStream_t);

}  // namespace tsfde
