// Full-dictionary OMP for dictionaries too large for the per-patch kernels.
#include <hip/hip_runtime.h>

#include "cspd_internal.h"

namespace cspd {

cspd_status launch_full_mfma(const cspd_plan_s *p, int64_t b, const void *y, const uint8_t *mask,
                             const int *kvec, int kuni, int *support, void *coef, int *k_used,
                             void *xhat, hipStream_t stream)
{
    (void)p; (void)b; (void)y; (void)mask; (void)kvec; (void)kuni; (void)support; (void)coef;
    (void)k_used; (void)xhat; (void)stream;
    return set_error(CSPD_E_UNSUPPORTED, "full search over %d atoms is not built yet", p->sc[p->s - 1].t);
}

}  // namespace cspd
