// LDS budget of the dense transform passes of the S_{n,S} and T_{n,S} block solvers (plain C++: the
// host check is tested on the CPU).  A pass keeps the transform's table (Np values: N for the Hartley
// transform, 2(N+1) for the sine transform) and up to kCasRows input rows of N values in dynamic LDS,
// and every launch also carries the kernel's static partial-sum array of 4 x kCasK values.
#pragma once

#include <algorithm>
#include <cstddef>

namespace tsfde {

constexpr int kCasK = 64;    // outputs per workgroup along the transformed index (one per lane)
constexpr int kCasRows = 4;  // rows per workgroup, one per wave
constexpr size_t kPassLdsBytes = 160 * 1024;

// dynamic LDS of one pass
inline size_t pass_dyn_lds(int N, int Np, int nrow, size_t elem) {
    return ((size_t)Np + (size_t)std::min(kCasRows, nrow) * (size_t)N) * elem;
}

// whole LDS of one pass: the dynamic part and the static partial sums
inline size_t pass_lds(int N, int Np, int nrow, size_t elem) {
    return pass_dyn_lds(N, Np, nrow, elem) + (size_t)4 * kCasK * elem;
}

// the passes of a d-dimensional block solve fit the LDS (FP64, the larger element)
inline bool dense_blocks_fit(int d, int N, int Np) {
    const int nrow = d == 2 ? N : 1;
    return N >= 1 && pass_lds(N, Np, nrow, sizeof(double)) <= kPassLdsBytes;
}

}  // namespace tsfde
