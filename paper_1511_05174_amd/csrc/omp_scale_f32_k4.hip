// Instantiations of the per-scale OMP kernel: float, up to 4 atoms per scale.
#include "omp_scale_impl.h"

namespace cspd {

cspd_status dispatch_scale_f32_k4(const ScaleArgs &a, int lp, int nc, int ppw, bool gram, bool mg,
                                     hipStream_t st)
{
    using namespace scale_impl;
    if (mg) {
        if (ppw == 2) {
            if (lp == 16) return launch_mg<16, 2, 4>(a, st);
            if (lp == 32) return launch_mg<32, 2, 4>(a, st);
            if (lp == 64) return launch_mg<64, 2, 4>(a, st);
            if (lp == 128) return launch_mg<128, 2, 4>(a, st);
        } else if (ppw == 1) {
            if (lp == 32) return launch_mg<32, 1, 4>(a, st);
            if (lp == 64) return launch_mg<64, 1, 4>(a, st);
            if (lp == 128) return launch_mg<128, 1, 4>(a, st);
        }
        return CSPD_E_UNSUPPORTED;
    }
    if (gram) {
        switch (nc) {
            case 1: return launch_one<float, 0, 1, 1, 4, true>(a, st);
            case 2: return launch_one<float, 0, 2, 1, 4, true>(a, st);
            case 4: return launch_one<float, 0, 4, 1, 4, true>(a, st);
            case 8: return launch_one<float, 0, 8, 1, 4, true>(a, st);
            case 16: return launch_one<float, 0, 16, 1, 4, true>(a, st);
            default: return CSPD_E_UNSUPPORTED;
        }
    }
    if (lp == 16 && nc == 1 && ppw == 2) return launch_one<float, 16, 1, 2, 4, false>(a, st);
    if (lp == 16 && nc == 2 && ppw == 2) return launch_one<float, 16, 2, 2, 4, false>(a, st);
    if (lp == 16 && nc == 4 && ppw == 2) return launch_one<float, 16, 4, 2, 4, false>(a, st);
    if (lp == 16 && nc == 4 && ppw == 1) return launch_one<float, 16, 4, 1, 4, false>(a, st);
    if (lp == 32 && nc == 1 && ppw == 2) return launch_one<float, 32, 1, 2, 4, false>(a, st);
    if (lp == 32 && nc == 2 && ppw == 2) return launch_one<float, 32, 2, 2, 4, false>(a, st);
    if (lp == 32 && nc == 2 && ppw == 1) return launch_one<float, 32, 2, 1, 4, false>(a, st);
    if (lp == 32 && nc == 4 && ppw == 1) return launch_one<float, 32, 4, 1, 4, false>(a, st);
    if (lp == 64 && nc == 1 && ppw == 2) return launch_one<float, 64, 1, 2, 4, false>(a, st);
    if (lp == 64 && nc == 1 && ppw == 1) return launch_one<float, 64, 1, 1, 4, false>(a, st);
    if (lp == 64 && nc == 2 && ppw == 1) return launch_one<float, 64, 2, 1, 4, false>(a, st);
    if (lp == 128 && nc == 1 && ppw == 1) return launch_one<float, 128, 1, 1, 4, false>(a, st);
    return CSPD_E_UNSUPPORTED;
}

}  // namespace cspd
