// Fixed-length instantiations of the tau-block form of the 2D segment kernel (T_{n,S}: every block
// solved by one application of its frozen-coefficient tau matrix) for N = 127, 255, 511.
#include "pinv_kernel.hpp"

namespace tsfde {

template <typename T>
bool launch_segments_fixed_tau(Problem& P, const Dev<T>& D, PersistentWork<T>& W, const T* z, T* y, bool last_block,
                               int blocks, hipStream_t st) {
    if (P.d != 2 || !P.tau_ok || P.Ld != P.L) return false;
    // no inner iterations, no warm start: tolerance, iteration cap and extrapolation are unused
    switch (P.L) {
        case 256:
            launch_segments<T, 8, SEG_2D_TAU, 256, true>(P, D, W, z, y, 0.0, 1, last_block, 0, blocks, st);
            return true;
        case 512:
            launch_segments<T, 8, SEG_2D_TAU, 512, true>(P, D, W, z, y, 0.0, 1, last_block, 0, blocks, st);
            return true;
        case 1024:
            launch_segments<T, 8, SEG_2D_TAU, 1024, true>(P, D, W, z, y, 0.0, 1, last_block, 0, blocks, st);
            return true;
        default:
            return false;
    }
}

template bool launch_segments_fixed_tau<double>(Problem&, const Dev<double>&, PersistentWork<double>&, const double*,
                                                double*, bool, int, hipStream_t);
template bool launch_segments_fixed_tau<float>(Problem&, const Dev<float>&, PersistentWork<float>&, const float*,
                                               float*, bool, int, hipStream_t);

}  // namespace tsfde
