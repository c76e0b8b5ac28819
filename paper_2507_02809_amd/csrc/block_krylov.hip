// Block flexible GMRES for several right-hand sides of the same all-at-once system (§5, eq. lin-syst):
// A X = B with X, B of p columns.  One block Krylov space serves all columns (the block GMRES of
// Saad, Iterative Methods for Sparse Linear Systems, in the chapter on Krylov methods for several
// right-hand sides); the preconditioner is applied column by column (flexible form, the directions
// Z_j = M V_j kept).  Each step:
//   W = A Z_j,                          Z_j = M V_j                 (p matvecs, p preconditioner calls)
//   H_{0:j,j} = V^T W, W -= V H, twice  (block classical Gram-Schmidt)
//   W = V_{j+1} H_{j+1,j}               (Cholesky QR, twice, columns scaled to unit norm first)
// and the block Hessenberg matrix is reduced by Givens rotations on the host, p rotations per column,
// so that the residual norm of every column is known after every step.
//
// The contractions V^T W and V H are matrix products with a dimension of n: they run on the FP64
// matrix cores (v_mfma_f64_16x16x4f64), 16 basis vectors by 16 columns per tile.  The basis is stored
// with a leading dimension rounded up to 64 doubles so that each vector starts 512-byte aligned.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "internal.hpp"

namespace tsfde {

typedef double bk_dbl4 __attribute__((ext_vector_type(4)));

constexpr int kBgChunk = 256;       // i values staged per workgroup step of the Gram kernel
constexpr int kBgPad = 17;          // LDS row length of the staged W^T (16 columns + 1)
constexpr int kBgMaxGrid = 2048;    // workgroups of a Gram launch (bounds the partial sums)

// ---------------------------------------------------------------------------
// G = V^T W (nv x p, p <= 16), partial sums per workgroup.  Workgroup (x, y): the basis vectors
// [16 TG x, 16 TG (x + 1)) against all columns, over the chunks [y cpb, (y + 1) cpb) of kBgChunk
// values of i.  W's chunk is staged in LDS transposed (wt[i][c]); wave w takes the four 16-value
// steps [4w, 4w + 4) of every chunk, and inside a step lane group q (= lane / 16) the four values
// i0 + 16u + 4q + e, e < 4, of its row (lane % 16), so that each row's 128 bytes are read by four
// lanes at once.  MFMA operands: A[row][q] = V[a0 + row][i], B[q][col] = W[col][i] with the same i
// in lane row + 16 q / col + 16 q; D[row][col] comes back in lane col + 16 (row % 4), value row / 4.
// The four waves' accumulators are added in LDS at the end.
// Rows past nv read row nv - 1 (in bounds) and are not written; V needs ldv % 4 == 0 and a 32-byte
// aligned base.
// ---------------------------------------------------------------------------
template <int TG>
__global__ __launch_bounds__(256) void bgram_k(const double* __restrict__ V, long long ldv, int nv,
                                               const double* __restrict__ W, long long ldw, int p, long long n,
                                               long long cpb, double* __restrict__ partials) {
    __shared__ double wt[kBgChunk * kBgPad];
    __shared__ double red[4][256];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = l >> 4, r16 = l & 15;
    const int a0 = blockIdx.x * TG * 16;
    const double* vrow[TG];
#pragma unroll
    for (int t = 0; t < TG; ++t) vrow[t] = V + (long long)min(a0 + t * 16 + r16, nv - 1) * ldv;
    bk_dbl4 acc[TG];
#pragma unroll
    for (int t = 0; t < TG; ++t) acc[t] = bk_dbl4{0.0, 0.0, 0.0, 0.0};
    const long long nch = (n + kBgChunk - 1) / kBgChunk;
    const long long c0 = (long long)blockIdx.y * cpb, c1 = min(nch, c0 + cpb);
    for (long long ch = c0; ch < c1; ++ch) {
        const long long i0 = ch * kBgChunk;
        __syncthreads();  // the previous chunk's readers are done with wt
        {
            const long long i = i0 + threadIdx.x;
            for (int c = 0; c < 16; ++c) wt[threadIdx.x * kBgPad + c] = (c < p && i < n) ? W[(long long)c * ldw + i] : 0.0;
        }
        __syncthreads();
        const bool full = i0 + kBgChunk <= n;
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) {
            const int ib = 16 * (w * 4 + uu) + 4 * q;  // offset of this lane's four values in the chunk
            double bv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) bv[e] = wt[(ib + e) * kBgPad + r16];
#pragma unroll
            for (int t = 0; t < TG; ++t) {
                double av[4];
                const double* src = vrow[t] + i0 + ib;
                if (full) {
                    const double2 lo = *reinterpret_cast<const double2*>(src);
                    const double2 hi = *reinterpret_cast<const double2*>(src + 2);
                    av[0] = lo.x;
                    av[1] = lo.y;
                    av[2] = hi.x;
                    av[3] = hi.y;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) av[e] = (i0 + ib + e < n) ? src[e] : 0.0;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[e], bv[e], acc[t], 0, 0, 0);
            }
        }
    }
    // add the four waves' tiles: element x = 64 v + lane of a tile is D[lane / 16 + 4 v][lane % 16]
#pragma unroll
    for (int t = 0; t < TG; ++t) {
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 4; ++v) red[w][v * 64 + l] = acc[t][v];
        __syncthreads();
        const int x = threadIdx.x;
        const double s = (red[0][x] + red[1][x]) + (red[2][x] + red[3][x]);
        const int lane = x & 63, v = x >> 6;
        const int a = a0 + t * 16 + (lane >> 4) + 4 * v;
        if (a < nv) partials[((long long)blockIdx.y * nv + a) * 16 + (lane & 15)] = s;
    }
}

// G[a][c] = sum over the y partial sums (a < nv, c < p; G row-major nv x p).  One wave per entry:
// lane l adds the partial sums y = l, l + 64, ... (their loads independent), then the 64 lane sums
// are added by a fixed shuffle tree, so the order is the same on every run.
__global__ __launch_bounds__(256) void bgram_finish_k(const double* __restrict__ partials, int ny, int nv, int p,
                                                      double* __restrict__ G) {
    const int l = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (idx >= nv * p) return;  // whole waves leave together
    const int a = idx / p, c = idx % p;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int y = l;
    for (; y + 192 < ny; y += 256)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += partials[((long long)(y + 64 * u) * nv + a) * 16 + c];
    for (; y < ny; y += 64) acc[0] += partials[((long long)y * nv + a) * 16 + c];
    double s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (l == 0) G[idx] = s;
}

// ---------------------------------------------------------------------------
// Y[c][i] = beta Y[c][i] + alpha sum_{a < nv} V[a][i] H[a][c]   (c < p <= 16, i < n)
// The product D = H^T V on the matrix cores: A[c][q] = H[a0 + q][c] (lane c + 16 q), B[q][i] =
// V[a0 + q][i] (lane i + 16 q, sixteen consecutive i per lane group: 128-byte reads), D[c][i] back in
// lane i + 16 (c % 4), value c / 4.  A wave covers NT tiles of 16 values of i.  Y may be V itself
// when nv == p: a wave reads all of its i range before it writes it, and waves own disjoint ranges.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(256) void bupdate_k(const double* V, long long ldv, int nv,
                                                 const double* __restrict__ H, int ldh, int p, double* Y,
                                                 long long ldy, long long n, double alpha, double beta) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = l >> 4, r16 = l & 15;
    const long long ib = ((long long)blockIdx.x * 4 + w) * (16 * NT);
    if (ib >= n) return;
    bk_dbl4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = bk_dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int a0 = 0; a0 < nv; a0 += 4) {
        const int a = a0 + q;
        const bool ok = a < nv;
        const double hv = (ok && r16 < p) ? H[(long long)a * ldh + r16] : 0.0;
        const double* vr = V + (long long)(ok ? a : nv - 1) * ldv + ib + r16;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bool in = ok && ib + t * 16 + r16 < n;
            const double bv = in ? vr[t * 16] : 0.0;
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(hv, bv, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const long long i = ib + t * 16 + r16;
        if (i >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = q + 4 * v;
            if (c < p) {
                double* y = Y + (long long)c * ldy + i;
                *y = beta != 0.0 ? beta * *y + alpha * acc[t][v] : alpha * acc[t][v];
            }
        }
    }
}

namespace {

long long round_ld(long long n) { return (n + 63) / 64 * 64; }

// G (host, nv x p row-major) = V^T W
void gram(Problem& P, const double* V, long long ldv, int nv, const double* W, long long ldw, int p,
          std::vector<double>& G, hipStream_t st) {
    const long long n = P.ntot;
    const long long nch = (n + kBgChunk - 1) / kBgChunk;
    const int tg = nv > 64 ? 8 : nv > 32 ? 4 : nv > 16 ? 2 : 1;
    const int gx = (nv + 16 * tg - 1) / (16 * tg);
    const long long ny0 = std::max<long long>(1, std::min<long long>(nch, kBgMaxGrid / gx));
    const long long cpb = (nch + ny0 - 1) / ny0;
    const int ny = (int)((nch + cpb - 1) / cpb);
    const dim3 grid((unsigned)gx, (unsigned)ny);
    switch (tg) {
        case 1: hipLaunchKernelGGL(bgram_k<1>, grid, dim3(256), 0, st, V, ldv, nv, W, ldw, p, n, cpb, P.blk_part); break;
        case 2: hipLaunchKernelGGL(bgram_k<2>, grid, dim3(256), 0, st, V, ldv, nv, W, ldw, p, n, cpb, P.blk_part); break;
        case 4: hipLaunchKernelGGL(bgram_k<4>, grid, dim3(256), 0, st, V, ldv, nv, W, ldw, p, n, cpb, P.blk_part); break;
        default: hipLaunchKernelGGL(bgram_k<8>, grid, dim3(256), 0, st, V, ldv, nv, W, ldw, p, n, cpb, P.blk_part); break;
    }
    TSFDE_HIP(hipGetLastError());
    hipLaunchKernelGGL(bgram_finish_k, dim3((nv * p + 3) / 4), dim3(256), 0, st, P.blk_part, ny, nv, p,
                       P.blk_small);
    TSFDE_HIP(hipGetLastError());
    G.resize((size_t)nv * p);
    TSFDE_HIP(hipMemcpyAsync(G.data(), P.blk_small, sizeof(double) * G.size(), hipMemcpyDeviceToHost, st));
    TSFDE_HIP(hipStreamSynchronize(st));
}

// Y = beta Y + alpha V H with H (host, nv x p row-major) uploaded first
void update(Problem& P, const double* V, long long ldv, int nv, const std::vector<double>& H, int p, double* Y,
            long long ldy, double alpha, double beta, hipStream_t st) {
    const long long n = P.ntot;
    TSFDE_HIP(hipMemcpyAsync(P.blk_small, H.data(), sizeof(double) * (size_t)nv * p, hipMemcpyHostToDevice, st));
    constexpr int NT = 4;
    const long long per_blk = 4LL * 16 * NT;
    const dim3 grid((unsigned)((n + per_blk - 1) / per_blk));
    hipLaunchKernelGGL(bupdate_k<NT>, grid, dim3(256), 0, st, V, ldv, nv, P.blk_small, p, p, Y, ldy, n, alpha, beta);
    TSFDE_HIP(hipGetLastError());
    // H's upload must not be overwritten before the kernel has read it
    TSFDE_HIP(hipStreamSynchronize(st));
}

// W (p columns, in place) = Q R: Cholesky QR of the column-scaled W, twice (R host, p x p row-major,
// upper).  A column whose part orthogonal to the earlier ones is below 1e-7 of its norm (pivot of the
// scaled Gram matrix <= kDefTol) is dependent: its column of Q is zero and its row of R is zero, and
// W = Q R holds to that level.  keep[c] tells which columns are independent; returns their number.
constexpr double kDefTol = 1e-14;

int chol_qr2(Problem& P, double* W, long long ldv, int p, std::vector<double>& R, std::vector<char>& keep,
             hipStream_t st) {
    std::vector<double> G, U((size_t)p * p), Ri((size_t)p * p), Rt, dsc(p);
    keep.assign(p, 1);
    R.assign((size_t)p * p, 0.0);
    for (int c = 0; c < p; ++c) R[(size_t)c * p + c] = 1.0;
    for (int pass = 0; pass < 2; ++pass) {
        gram(P, W, ldv, p, W, ldv, p, G, st);
        for (int c = 0; c < p; ++c) {
            const double g = G[(size_t)c * p + c];
            dsc[c] = g > 0.0 ? std::sqrt(g) : 1.0;
        }
        // Cholesky of D^-1 G D^-1 = U^T U, a dependent column leaving a zero row of U
        std::fill(U.begin(), U.end(), 0.0);
        for (int i = 0; i < p; ++i) {
            double s = G[(size_t)i * p + i] / (dsc[i] * dsc[i]);
            for (int k = 0; k < i; ++k) s -= U[(size_t)k * p + i] * U[(size_t)k * p + i];
            if (!(s > kDefTol)) {
                keep[i] = 0;
                continue;
            }
            const double uii = std::sqrt(s);
            U[(size_t)i * p + i] = uii;
            for (int j = i + 1; j < p; ++j) {
                double t = G[(size_t)i * p + j] / (dsc[i] * dsc[j]);
                for (int k = 0; k < i; ++k) t -= U[(size_t)k * p + i] * U[(size_t)k * p + j];
                U[(size_t)i * p + j] = t / uii;
            }
        }
        // this pass's factor U D and the inverse of its independent part (zero elsewhere)
        for (int i = 0; i < p; ++i)
            for (int j = i; j < p; ++j) U[(size_t)i * p + j] *= dsc[j];
        std::fill(Ri.begin(), Ri.end(), 0.0);
        for (int j = 0; j < p; ++j) {
            if (!keep[j]) continue;
            for (int i = j; i >= 0; --i) {
                if (!keep[i]) continue;
                double t = i == j ? 1.0 : 0.0;
                for (int k = i + 1; k <= j; ++k)
                    if (keep[k]) t -= U[(size_t)i * p + k] * Ri[(size_t)k * p + j];
                Ri[(size_t)i * p + j] = t / U[(size_t)i * p + i];
            }
        }
        update(P, W, ldv, p, Ri, p, W, ldv, 1.0, 0.0, st);
        Rt.assign((size_t)p * p, 0.0);
        for (int i = 0; i < p; ++i)
            for (int j = i; j < p; ++j) {
                double t = 0.0;
                for (int k = i; k <= j; ++k) t += U[(size_t)i * p + k] * R[(size_t)k * p + j];
                Rt[(size_t)i * p + j] = t;
            }
        R.swap(Rt);
    }
    int r = 0;
    for (int c = 0; c < p; ++c) r += keep[c] ? 1 : 0;
    return r;
}

// a residual norm, NaN kept (so that a NaN never reads as converged)
double safe_sqrt(double g) { return g < 0.0 ? 0.0 : std::sqrt(g); }

}  // namespace

size_t block_basis_bytes(const Problem& P, int p, int m) {
    return sizeof(double) * (size_t)round_ld(P.ntot) * (size_t)((m + 1) * p + m * p);
}

// The basis V ((m + 1) p vectors) and the directions Z (m p vectors), leading dimension ldv, the
// Gram partial sums and a small transfer buffer (allocated on first use, grown as needed).
static long long ensure_block_basis(Problem& P, int p, int m, const Opts& o) {
    const long long ldv = round_ld(P.ntot);
    const size_t need = block_basis_bytes(P, p, m);
    if (P.blk_nvec >= (m + 1) * p + m * p && P.blk_p == p) return ldv;
    if (o.max_device_bytes > 0 && P.bytes - P.blk_bytes + need > (size_t)o.max_device_bytes) {
        char buf[256];
        std::snprintf(buf, sizeof(buf),
                      "max_device_bytes = %lld: the problem holds %zu bytes and the block basis of %d columns and "
                      "restart %d needs %zu more",
                      o.max_device_bytes, P.bytes - P.blk_bytes, p, m, need);
        throw CapError{buf};
    }
    if (P.blk_V) (void)hipFree(P.blk_V);
    P.blk_V = nullptr;
    P.bytes -= P.blk_bytes;
    P.blk_bytes = 0;
    P.blk_nvec = 0;
    const size_t nvec = (size_t)((m + 1) * p + m * p);
    dev_alloc(P, P.blk_V, nvec * (size_t)ldv);
    P.blk_bytes = need;
    P.blk_nvec = (int)nvec;
    P.blk_p = p;
    if (!P.blk_part) dev_alloc(P, P.blk_part, (size_t)kBgMaxGrid * 128 * 16);
    if (!P.blk_small) dev_alloc(P, P.blk_small, (size_t)kBlockMaxBasis * 16);
    return ldv;
}

int block_fgmres(Problem& P, const SolveOps& ops, int p, const double* B, double* X, double rtol, int restart,
                 int maxit, hipStream_t st, tsfde_stats& S, std::vector<double>& rel, bool& conv, const Opts& o) {
    const long long n = P.ntot;
    const int m = restart;
    const long long ldv = ensure_block_basis(P, p, m, o);
    double* V = P.blk_V;                                  // up to (m + 1) p vectors
    double* Z = P.blk_V + (size_t)(m + 1) * p * ldv;      // up to m p vectors
    auto vcol = [&](int a) { return V + (size_t)a * ldv; };
    auto zcol = [&](int a) { return Z + (size_t)a * ldv; };
    std::vector<double> bnorm(p), G, R, S0, Hb, Gl, Y, H1, H2;
    std::vector<char> keep;
    std::vector<int> rot_row;
    std::vector<double> rot_c, rot_s;
    rel.assign(p, 1.0);
    conv = false;
    // ||b_c|| from the Gram matrix of B copied into the basis
    for (int c = 0; c < p; ++c) launch_copy<double>(B + (size_t)c * n, vcol(c), n, st);
    gram(P, V, ldv, p, V, ldv, p, G, st);
    for (int c = 0; c < p; ++c) bnorm[c] = safe_sqrt(G[(size_t)c * p + c]);
    auto scaled = [&](int c, double r) { return bnorm[c] > 0.0 ? r / bnorm[c] : r; };
    auto largest = [&]() {
        double w = 0.0;
        for (int c = 0; c < p; ++c)
            if (!(rel[c] <= w)) w = rel[c];  // NaN wins
        return w;
    };
    int its = 0;
    while (true) {
        // R0 = B - A X in the basis, its true column norms
        double t0 = now_seconds();
        for (int c = 0; c < p; ++c) ops.A(X + (size_t)c * n, vcol(c));
        TSFDE_HIP(hipStreamSynchronize(st));
        S.t_matvec += now_seconds() - t0;
        for (int c = 0; c < p; ++c) launch_axpby(1.0, B + (size_t)c * n, -1.0, vcol(c), vcol(c), n, st);
        gram(P, V, ldv, p, V, ldv, p, G, st);
        for (int c = 0; c < p; ++c) rel[c] = scaled(c, safe_sqrt(G[(size_t)c * p + c]));
        double worst = largest();
        P.res_hist.push_back(worst);
        if (worst <= rtol) {
            conv = true;
            break;
        }
        if (its >= maxit || std::isnan(worst)) break;
        // R0 = V0 S0; the block keeps only R0's independent columns (s of them), so the block width s
        // of this cycle may be below p, while S0's rows still carry all p right-hand sides
        t0 = now_seconds();
        const int s = chol_qr2(P, V, ldv, p, S0, keep, st);
        if (s == 0) break;
        {
            int t = 0;
            for (int c = 0; c < p; ++c)
                if (keep[c]) {
                    if (t != c) launch_copy<double>(vcol(c), vcol(t), n, st);
                    for (int cc = 0; cc < p; ++cc) S0[(size_t)t * p + cc] = S0[(size_t)c * p + cc];
                    ++t;
                }
        }
        S.t_ortho += now_seconds() - t0;
        const int mm = std::min(m, maxit - its);
        const int rows = (mm + 1) * s, cols = mm * s;
        Hb.assign((size_t)rows * cols, 0.0);
        Gl.assign((size_t)rows * p, 0.0);
        for (int i = 0; i < s; ++i)
            for (int c = 0; c < p; ++c) Gl[(size_t)i * p + c] = S0[(size_t)i * p + c];
        rot_row.clear();
        rot_c.clear();
        rot_s.clear();
        int k = 0;
        for (int j = 0; j < mm; ++j) {
            const int nv = (j + 1) * s;
            double* Wb = vcol(nv);
            t0 = now_seconds();
            for (int c = 0; c < s; ++c) S.inner_iters += ops.M(vcol(j * s + c), zcol(j * s + c));
            TSFDE_HIP(hipStreamSynchronize(st));
            S.t_precond += now_seconds() - t0;
            t0 = now_seconds();
            for (int c = 0; c < s; ++c) ops.A(zcol(j * s + c), vcol(nv + c));
            TSFDE_HIP(hipStreamSynchronize(st));
            S.t_matvec += now_seconds() - t0;
            t0 = now_seconds();
            // block classical Gram-Schmidt, twice, then W = V_{j+1} R
            gram(P, V, ldv, nv, Wb, ldv, s, H1, st);
            update(P, V, ldv, nv, H1, s, Wb, ldv, -1.0, 1.0, st);
            gram(P, V, ldv, nv, Wb, ldv, s, H2, st);
            update(P, V, ldv, nv, H2, s, Wb, ldv, -1.0, 1.0, st);
            const int r = chol_qr2(P, Wb, ldv, s, R, keep, st);
            S.t_ortho += now_seconds() - t0;
            for (int i = 0; i < nv; ++i)
                for (int c = 0; c < s; ++c) Hb[(size_t)i * cols + j * s + c] = H1[(size_t)i * s + c] + H2[(size_t)i * s + c];
            for (int i = 0; i < s; ++i)
                for (int c = i; c < s; ++c) Hb[(size_t)(nv + i) * cols + j * s + c] = R[(size_t)i * s + c];
            // Givens: the earlier rotations on the new columns, then s new ones per column
            for (int c = 0; c < s; ++c) {
                const int qc = j * s + c;
                for (size_t t = 0; t < rot_row.size(); ++t) {
                    const int i = rot_row[t];
                    const double a = Hb[(size_t)i * cols + qc], b = Hb[(size_t)(i + 1) * cols + qc];
                    Hb[(size_t)i * cols + qc] = rot_c[t] * a + rot_s[t] * b;
                    Hb[(size_t)(i + 1) * cols + qc] = -rot_s[t] * a + rot_c[t] * b;
                }
                for (int i = qc + s; i > qc; --i) {
                    const double a = Hb[(size_t)(i - 1) * cols + qc], b = Hb[(size_t)i * cols + qc];
                    const double rr = std::hypot(a, b);
                    const double cs = rr > 0.0 ? a / rr : 1.0, sn = rr > 0.0 ? b / rr : 0.0;
                    Hb[(size_t)(i - 1) * cols + qc] = rr;
                    Hb[(size_t)i * cols + qc] = 0.0;
                    for (int cc = 0; cc < p; ++cc) {
                        const double ga = Gl[(size_t)(i - 1) * p + cc], gb = Gl[(size_t)i * p + cc];
                        Gl[(size_t)(i - 1) * p + cc] = cs * ga + sn * gb;
                        Gl[(size_t)i * p + cc] = -sn * ga + cs * gb;
                    }
                    rot_row.push_back(i - 1);
                    rot_c.push_back(cs);
                    rot_s.push_back(sn);
                }
            }
            k = j + 1;
            ++its;
            ++S.iters;
            // residual of right-hand side c: rows [(j + 1) s, (j + 2) s) of the rotated G
            for (int c = 0; c < p; ++c) {
                double t = 0.0;
                for (int i = nv; i < nv + s; ++i) t += Gl[(size_t)i * p + c] * Gl[(size_t)i * p + c];
                rel[c] = scaled(c, std::sqrt(t));
            }
            worst = largest();
            P.res_hist.push_back(worst);
            if (worst <= rtol || its >= maxit || std::isnan(worst)) break;
            // a dependent column in W: the block Krylov space is (nearly) invariant in that direction;
            // the cycle ends here and the restart continues from the true residual
            if (r < s) break;
        }
        // Y = R^{-1} G over the k s columns, X += Z Y
        const int ks = k * s;
        Y.assign((size_t)ks * p, 0.0);
        for (int c = 0; c < p; ++c)
            for (int i = ks - 1; i >= 0; --i) {
                double t = Gl[(size_t)i * p + c];
                for (int l = i + 1; l < ks; ++l) t -= Hb[(size_t)i * cols + l] * Y[(size_t)l * p + c];
                const double d = Hb[(size_t)i * cols + i];
                Y[(size_t)i * p + c] = d != 0.0 ? t / d : 0.0;
            }
        t0 = now_seconds();
        update(P, Z, ldv, ks, Y, p, X, n, 1.0, 1.0, st);
        S.t_ortho += now_seconds() - t0;
        ++S.restarts;
    }
    return its;
}

}  // namespace tsfde
