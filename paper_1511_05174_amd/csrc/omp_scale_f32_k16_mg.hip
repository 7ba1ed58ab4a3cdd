// Instantiations of the per-scale OMP kernel: float, up to 16 atoms per scale,
// candidate Gram matrices on the matrix cores.  Built with the iteration loop
// fully unrolled (its trip count is bounded by 16 but has an early exit), so
// that every iteration's dot products stop at the rows filled so far.
#include "omp_scale_impl.h"

namespace cspd {

cspd_status dispatch_scale_f32_k16_mg(const ScaleArgs &a, int lp, int ppw, hipStream_t st)
{
    using namespace scale_impl;
    if (ppw == 2) {
        if (lp == 16) return launch_mg<16, 2, 16>(a, st);
        if (lp == 32) return launch_mg<32, 2, 16>(a, st);
        if (lp == 64) return launch_mg<64, 2, 16>(a, st);
        if (lp == 128) return launch_mg<128, 2, 16>(a, st);
    } else if (ppw == 1) {
        if (lp == 32) return launch_mg<32, 1, 16>(a, st);
        if (lp == 64) return launch_mg<64, 1, 16>(a, st);
        if (lp == 128) return launch_mg<128, 1, 16>(a, st);
    }
    return CSPD_E_UNSUPPORTED;
}

}  // namespace cspd
