// Shared device/host helpers for the tsfde library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tsfde {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }

constexpr int kWave = 64;

// Deterministic block reduction of one value per thread; result valid in thread 0.
// `smem` must hold blockDim.x / 64 doubles.
// Works for any blockDim.x <= 256, including partially filled waves.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* smem) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nact = min(kWave, (int)blockDim.x - wid * kWave);  // active lanes of this wave
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const T o = __shfl_down(v, off, kWave);
        if (lane + off < nact) v += o;
    }
    if (lane == 0) smem[wid] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + kWave - 1) / kWave;
        for (int w = 0; w < nw; ++w) r += smem[w];
    }
    __syncthreads();
    return r;
}

inline int ilog2(long long v) {
    int r = 0;
    while ((1LL << r) < v) ++r;
    return r;
}

inline bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace tsfde
