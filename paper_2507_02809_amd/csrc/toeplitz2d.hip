// Matvec Toeplitz product for d = 2 (§5 matvec step 1(b): embed B_n in a two-level circulant,
// FFT, multiply by the circulant's eigenvalues, inverse FFT, crop), arranged for streaming all
// M+1 slices of a vector through HBM:
//
//   rows_fwd : a workgroup of gpb transform groups takes 2 gpb consecutive rows of one slice
//              (group g: rows i0 = ibase + 2g and i0 + 1, packed as one complex sequence), loads
//              them straight into the FFT's register layout, transforms, and the whole workgroup
//              writes the two half spectra transposed, spec[slice][k2][i] (k2 <= L/2, row
//              stride ns), two adjacent i per thread so that a wave covers 2 gpb consecutive i
//              of 16 rows k2;
//   cols     : one group per spectral row (slice, k2): zero-padded FFT over i, times the symbol
//              lambda(k1, k2)/L^2, inverse FFT, first N values back; both transforms stay in
//              registers apart from their internal exchanges;
//   rows_inv : the workgroup loads the half spectra of its 2 gpb rows (same coalesced pattern),
//              each group re-packs its pair into one Hermitian-completed spectrum, the inverse
//              FFT leaves the pair's rows in registers, and the epilogue adds c_t gamma2 .* (B y)
//              to the history part already in z (slice s < M), or writes
//              z_M = c_f gamma2_{M-1} .* (B f) + ylast, ylast = y_{M-1} for A (a null gamma2
//              stands for ones: the transposed operator applies B to gamma2-scaled slices).
//
// The transform length is a template constant for L = 512 (the C3 size), a run-time value
// otherwise.  Requires N <= L/2 (the embedding has L >= 2N).
#include <cstdlib>

#include "fft.hpp"
#include "internal.hpp"

namespace tsfde {

constexpr int kMvBlock = 256;

__host__ __device__ constexpr int mv_stride(int N) { return (N + 15) & ~15; }

template <typename T, int VPT, int LC>
__global__ __launch_bounds__(kMvBlock) void mv_rows_fwd(const T* __restrict__ y, int N, int L_, int nsl,
                                                        const cplx<T>* __restrict__ tw_g, cplx<T>* __restrict__ spec) {
    extern __shared__ unsigned char smem_raw[];
    const int L = LC ? LC : L_;
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);  // twiddle table, then the groups' sequences
    cplx<T>* cbase = tw + L;
    const int H = L / 2 + 1, LP = lds_len(L), ns = mv_stride(N);
    const int nthr = L / VPT, gpb = kMvBlock / nthr;
    const int grp = threadIdx.x / nthr, tid = threadIdx.x - grp * nthr;
    const int nrb = (N + 2 * gpb - 1) / (2 * gpb);
    const long long Nd = (long long)N * N;
    for (int k = threadIdx.x; k < L; k += kMvBlock) tw[k] = tw_g[k];
    __syncthreads();
    cplx<T>* c = cbase + (size_t)grp * LP;
    constexpr int VH = VPT / 2;  // j < N <= L/2 = VH * nthr
    // the rows of the next block are loaded while the current block is transformed (barriers wait
    // for LDS operations only, so the loads stay in flight)
    T p0[VH], p1[VH];
    auto load_rows = [&](int b) {
        const int sl = b / nrb;
        const int i0 = (b - sl * nrb) * 2 * gpb + 2 * grp;
        const T* ys = y + (long long)sl * Nd;
#pragma unroll
        for (int u = 0; u < VH; ++u) {
            const int j = tid + u * nthr;
            p0[u] = p1[u] = T(0);
            if (j < N && i0 < N) {
                p0[u] = ys[(long long)i0 * N + j];
                if (i0 + 1 < N) p1[u] = ys[(long long)(i0 + 1) * N + j];
            }
        }
    };
    if (blockIdx.x < nrb * nsl) load_rows(blockIdx.x);
    for (int blk = blockIdx.x; blk < nrb * nsl; blk += gridDim.x) {  // uniform per workgroup
        const int slice = blk / nrb;
        const int ibase = (blk - slice * nrb) * 2 * gpb;
        cplx<T> v[VPT];
#pragma unroll
        for (int u = 0; u < VPT; ++u) v[u] = (u < VH) ? cplx<T>{p0[u], p1[u]} : cplx<T>{T(0), T(0)};
        if (blk + (int)gridDim.x < nrb * nsl) load_rows(blk + gridDim.x);
        fft_x<T, VPT, false, true, false>(v, c, L, tw, tid, nthr);
        __syncthreads();  // the write-out reads every group's sequence
        cplx<T>* out = spec + (long long)slice * H * ns;
        for (int idx = threadIdx.x; idx < H * gpb; idx += kMvBlock) {
            const int k = idx / gpb, g = idx - k * gpb;
            const int i = ibase + 2 * g;
            if (i >= N) continue;
            const cplx<T>* cg = cbase + (size_t)g * LP;
            const cplx<T> C = cg[lx(k)];
            const cplx<T> Cm = cg[lx((L - k) & (L - 1))];
            cplx<T>* dst = out + (long long)k * ns + i;
            dst[0] = {T(0.5) * (C.x + Cm.x), T(0.5) * (C.y - Cm.y)};
            if (i + 1 < N) dst[1] = {T(0.5) * (C.y + Cm.y), T(0.5) * (Cm.x - C.x)};
        }
        __syncthreads();  // the sequences are free for the next rows
    }
}

template <typename T, int VPT, int LC>
__global__ __launch_bounds__(kMvBlock) void mv_cols(cplx<T>* __restrict__ spec, int N, int L_, int nrows,
                                                    const cplx<T>* __restrict__ tw_g, const T* __restrict__ sym) {
    // the twiddle table sits in LDS in front of the groups' sequences; each workgroup walks over
    // several spectral rows so that the table is loaded once per workgroup
    extern __shared__ unsigned char smem_raw[];
    const int L = LC ? LC : L_;
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* cbase = tw + L;
    const int H = L / 2 + 1, LP = lds_len(L), ns = mv_stride(N);
    const int nthr = L / VPT, gpb = kMvBlock / nthr;
    const int grp = threadIdx.x / nthr, tid = threadIdx.x - grp * nthr;
    for (int k = threadIdx.x; k < L; k += kMvBlock) tw[k] = tw_g[k];
    __syncthreads();
    cplx<T>* c = cbase + (size_t)grp * LP;
    constexpr int VH = VPT / 2;
    const int stride = gridDim.x * gpb;
    const int rounds = (nrows + stride - 1) / stride;  // the same for every group (the FFTs hold barriers)
    // the next round's row and symbol are loaded while the current row is transformed (barriers
    // wait for LDS operations only, so the loads stay in flight)
    cplx<T> pv[VH];
    T ps[VPT];
    auto load_row = [&](int r) {
        const int rowid = r * stride + blockIdx.x * gpb + grp;  // (slice, k2) flattened, slice-major
        const bool ok = rowid < nrows;
        const int sl = ok ? rowid / H : 0;
        const int kk = ok ? rowid - sl * H : 0;
        const cplx<T>* rw = spec + ((long long)sl * H + kk) * ns;
        const T* sy = sym + (long long)kk * L;
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int i = tid + u * nthr;
            if (u < VH) pv[u] = (ok && i < N) ? rw[i] : cplx<T>{T(0), T(0)};
            ps[u] = sy[i];
        }
    };
    if (rounds > 0) load_row(0);
    for (int rd = 0; rd < rounds; ++rd) {
        const int rowid = rd * stride + blockIdx.x * gpb + grp;  // (slice, k2) flattened, slice-major
        const bool valid = rowid < nrows;
        const int slice = valid ? rowid / H : 0;
        const int k2 = valid ? rowid - slice * H : 0;
        cplx<T>* row = spec + ((long long)slice * H + k2) * ns;
        cplx<T> v[VPT];
        T sv[VPT];
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            v[u] = (u < VH) ? pv[u] : cplx<T>{T(0), T(0)};
            sv[u] = ps[u];
        }
        if (rd + 1 < rounds) load_row(rd + 1);
        fft_x<T, VPT, false, true, true>(v, c, L, tw, tid, nthr);
#pragma unroll
        for (int u = 0; u < VPT; ++u) v[u] = {v[u].x * sv[u], v[u].y * sv[u]};
        fft_x<T, VPT, true, true, true>(v, c, L, tw, tid, nthr);
        if (valid) {
#pragma unroll
            for (int u = 0; u < VH; ++u) {
                const int i = tid + u * nthr;
                if (i < N) row[i] = v[u];
            }
        }
    }
}

template <typename T, int VPT, int LC>
__global__ __launch_bounds__(kMvBlock) void mv_rows_inv(const cplx<T>* __restrict__ spec, int N, int L_, int slice0,
                                                        int nsl, int M, const cplx<T>* __restrict__ tw_g,
                                                        T* __restrict__ z, const T* __restrict__ ylast,
                                                        const T* __restrict__ g2, T ct, T cf) {
    extern __shared__ unsigned char smem_raw[];
    const int L = LC ? LC : L_;
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);  // twiddle table, then the groups' sequences
    cplx<T>* cbase = tw + L;
    const int H = L / 2 + 1, LP = lds_len(L), ns = mv_stride(N);
    const int nthr = L / VPT, gpb = kMvBlock / nthr;
    const int grp = threadIdx.x / nthr, tid = threadIdx.x - grp * nthr;
    const int nrb = (N + 2 * gpb - 1) / (2 * gpb);
    const long long Nd = (long long)N * N;
    for (int k = threadIdx.x; k < L; k += kMvBlock) tw[k] = tw_g[k];
    __syncthreads();
    cplx<T>* c = cbase + (size_t)grp * LP;
    constexpr int VH = VPT / 2;
    for (int blk = blockIdx.x; blk < nrb * nsl; blk += gridDim.x) {  // uniform per workgroup
        const int sl = blk / nrb;
        const int ibase = (blk - sl * nrb) * 2 * gpb;
        const int i0 = ibase + 2 * grp;
        const bool two = i0 + 1 < N;
        const int s = slice0 + sl;
        const bool last = (s == M);
        // epilogue operands first (their latency overlaps the spectrum loads and the transform)
        T zo0[VH], zo1[VH], gv0[VH], gv1[VH];
#pragma unroll
        for (int u = 0; u < VH; ++u) {
            const int j = tid + u * nthr;
            zo0[u] = zo1[u] = gv0[u] = gv1[u] = T(0);
            if (j < N && i0 < N) {
                const long long o = (long long)i0 * N + j;
                const long long gs = (long long)(last ? M - 1 : s) * Nd;
                gv0[u] = g2 ? g2[gs + o] : T(1);
                zo0[u] = last ? ylast[o] : z[(long long)s * Nd + o];
                if (two) {
                    gv1[u] = g2 ? g2[gs + o + N] : T(1);
                    zo1[u] = last ? ylast[o + N] : z[(long long)s * Nd + o + N];
                }
            }
        }
        const cplx<T>* sp = spec + (long long)sl * H * ns;
        for (int idx = threadIdx.x; idx < H * gpb; idx += kMvBlock) {
            const int k = idx / gpb, g = idx - k * gpb;
            const int i = ibase + 2 * g;
            cplx<T> Y0 = {T(0), T(0)}, Y1 = {T(0), T(0)};
            if (i < N) {
                const cplx<T>* src = sp + (long long)k * ns + i;
                Y0 = src[0];
                if (i + 1 < N) Y1 = src[1];
            }
            cplx<T>* cg = cbase + (size_t)g * LP;
            cg[lx(k)] = {Y0.x - Y1.y, Y0.y + Y1.x};
            if (k > 0 && k < H - 1) cg[lx(L - k)] = {Y0.x + Y1.y, Y1.x - Y0.y};
        }
        __syncthreads();
        cplx<T> v[VPT];
        fft_x<T, VPT, true, false, true>(v, c, L, tw, tid, nthr);  // ends with the sequences free
        const T cc = last ? cf : ct;
#pragma unroll
        for (int u = 0; u < VH; ++u) {
            const int j = tid + u * nthr;
            if (j < N && i0 < N) {
                const long long o = (long long)s * Nd + (long long)i0 * N + j;
                z[o] = zo0[u] + cc * gv0[u] * v[u].x;
                if (two) z[o + N] = zo1[u] + cc * gv1[u] * v[u].y;
            }
        }
    }
}

template <typename T, int VPT, int LC>
static void launch_mv(const Problem& P, const Dev<T>& D, const T* y, T* z, const T* ylast, hipStream_t st,
                      hipEvent_t before_inv) {
    const int L = P.L, N = P.N, H = L / 2 + 1;
    const int nthr = L / VPT, gpb = kMvBlock / nthr;
    const size_t lds = sizeof(cplx<T>) * ((size_t)L + (size_t)gpb * lds_len(L));  // twiddles + sequences
    const int nslices = P.M + 1;
    const int nrb = (N + 2 * gpb - 1) / (2 * gpb);
    // workgroups loop over the work (the twiddle table is loaded once each): one full wave of
    // resident workgroups per kernel
    thread_local int res[3] = {0, 0, 0};
    thread_local size_t res_lds = 0;  // occupancy depends on the LDS size (L is a run-time value for LC = 0)
    if (res_lds != lds) {
        res_lds = lds;
        int dev = 0, ncu = 0;
        TSFDE_HIP(hipGetDevice(&dev));
        TSFDE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        int b0 = 0, b1 = 0, b2 = 0;
        TSFDE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b0, mv_rows_fwd<T, VPT, LC>, kMvBlock, lds));
        TSFDE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, mv_cols<T, VPT, LC>, kMvBlock, lds));
        TSFDE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, mv_rows_inv<T, VPT, LC>, kMvBlock, lds));
        res[1] = std::max(1, b1) * ncu;
        res[2] = std::max(1, b2) * ncu;
        res[0] = std::max(1, b0) * ncu;
    }
    // TSFDE_MV_CHUNK (diagnostics): slices per pass of the three kernels
    int chunk = P.nspec;
    if (const char* e = std::getenv("TSFDE_MV_CHUNK")) chunk = std::max(1, std::min(P.nspec, std::atoi(e)));
    for (int s0 = 0; s0 < nslices; s0 += chunk) {
        const int nsl = std::min(chunk, nslices - s0);
        const T* ys = y + (long long)s0 * P.Nd;
        hipLaunchKernelGGL((mv_rows_fwd<T, VPT, LC>), dim3(std::min(nrb * nsl, res[0])), dim3(kMvBlock), lds, st, ys,
                           N, L, nsl, D.tw, D.spec);
        const int nrows = nsl * H;
        hipLaunchKernelGGL((mv_cols<T, VPT, LC>), dim3(std::min((nrows + gpb - 1) / gpb, res[1])), dim3(kMvBlock), lds,
                           st, D.spec, N, L, nrows, D.tw, D.sym);
        // the epilogue adds to z: whatever else writes z (the history sum on another stream) first
        if (before_inv && s0 == 0) TSFDE_HIP(hipStreamWaitEvent(st, before_inv, 0));
        hipLaunchKernelGGL((mv_rows_inv<T, VPT, LC>), dim3(std::min(nrb * nsl, res[2])), dim3(kMvBlock), lds, st,
                           D.spec, N, L, s0, nsl, P.M, D.tw, z, ylast, D.gamma2, T(P.ct), T(P.cf));
        TSFDE_HIP(hipGetLastError());
    }
}

bool toeplitz2d_supported(const Problem& P) { return P.d == 2 && 2 * P.N <= P.L && P.L >= 16 && P.L <= 4096; }

template <typename T>
bool launch_toeplitz2d_matvec(const Problem& P, const Dev<T>& D, const T* y, T* z, hipStream_t st,
                              const T* ylast, hipEvent_t before_inv) {
    if (!toeplitz2d_supported(P)) return false;
    const int L = P.L;
    if (!ylast) ylast = y + (long long)(P.M - 1) * P.Nd;
    // TSFDE_MV_VARIANT (diagnostics) overrides the problem's tuned tiling
    int v = P.mv_variant;
    if (const char* e = std::getenv("TSFDE_MV_VARIANT")) v = std::atoi(e);
    if (v < 0) v = L == 512 ? 0 : (L <= 2048 ? 1 : 2);  // built-in choice
    switch (v) {
        case 0: launch_mv<T, 8, 512>(P, D, y, z, ylast, st, before_inv); break;
        case 1: launch_mv<T, 8, 0>(P, D, y, z, ylast, st, before_inv); break;
        case 2: launch_mv<T, 16, 0>(P, D, y, z, ylast, st, before_inv); break;
        case 3: launch_mv<T, 32, 0>(P, D, y, z, ylast, st, before_inv); break;
        case 4: launch_mv<T, 16, 512>(P, D, y, z, ylast, st, before_inv); break;
        default: throw HipError{hipErrorInvalidValue, "2D matvec: unknown FFT tiling"};
    }
    return true;
}

int mv_variants(const Problem& P, int* ids, int max_ids) {
    if (!toeplitz2d_supported(P)) return 0;
    const int L = P.L;
    const int vpt[5] = {8, 8, 16, 32, 16};
    const bool fixed[5] = {true, false, false, false, true};
    int n = 0;
    for (int v = 0; v < 5 && n < max_ids; ++v) {
        if (fixed[v] && L != 512) continue;
        const int nthr = L / vpt[v];
        if (nthr < 8 || nthr > kMvBlock) continue;
        const int gpb = kMvBlock / nthr;
        const size_t lds = sizeof(cplx<double>) * ((size_t)L + (size_t)gpb * lds_len(L));
        if (lds > 160 * 1024) continue;
        ids[n++] = v;
    }
    return n;
}

template bool launch_toeplitz2d_matvec<double>(const Problem&, const Dev<double>&, const double*, double*,
                                               hipStream_t, const double*, hipEvent_t);
template bool launch_toeplitz2d_matvec<float>(const Problem&, const Dev<float>&, const float*, float*, hipStream_t,
                                              const float*, hipEvent_t);

}  // namespace tsfde
