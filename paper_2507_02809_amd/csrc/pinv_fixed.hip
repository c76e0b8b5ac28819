// Fixed-length instantiations of the 2D sine-transform segment kernel (the transform length L,
// and with it N = L/2 - 1, a compile-time constant) for the common grid sizes N = 127, 255, 511.
#include "pinv_kernel.hpp"

namespace tsfde {

template <typename T>
bool launch_segments_fixed(Problem& P, const Dev<T>& D, PersistentWork<T>& W, const T* z, T* y, double inner_tol,
                           int inner_maxit, bool last_block, int extrap, int blocks, hipStream_t st) {
    if (P.d != 2 || !P.tau_ok || P.Ld != P.L) return false;
    switch (P.L) {
        case 256:
            launch_segments<T, 8, SEG_2D_TAU, 256, false>(P, D, W, z, y, inner_tol, inner_maxit, last_block, extrap, blocks, st);
            return true;
        case 512:
            launch_segments<T, 8, SEG_2D_TAU, 512, false>(P, D, W, z, y, inner_tol, inner_maxit, last_block, extrap, blocks, st);
            return true;
        case 1024:
            launch_segments<T, 8, SEG_2D_TAU, 1024, false>(P, D, W, z, y, inner_tol, inner_maxit, last_block, extrap, blocks, st);
            return true;
        default:
            return false;
    }
}

template bool launch_segments_fixed<double>(Problem&, const Dev<double>&, PersistentWork<double>&, const double*,
                                            double*, double, int, bool, int, int, hipStream_t);
template bool launch_segments_fixed<float>(Problem&, const Dev<float>&, PersistentWork<float>&, const float*, float*,
                                           double, int, bool, int, int, hipStream_t);

}  // namespace tsfde
