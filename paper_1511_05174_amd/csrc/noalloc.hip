// Zero-tree OMP for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The cross-scale call's only device memory beyond the caller's inputs and
// outputs is its workspace: the coarse scales' k_used, their supports unless
// the caller keeps them, and scale 0's correlations on the dense-operator GEMM
// path.  Here that workspace is a fixed array in device memory, one copy per
// GPU, reserved when the code object loads and held until the process ends.
// Every kernel writes the workspace entries it later reads (each scale writes
// all k_used entries and all support slots of its patches before the next
// scale reads them), so nothing has to start at zero.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cspd_internal.h"

namespace cspd {

namespace {

// The workspace.  In host code `scratch` names a host-side stand-in, not the
// device array: its device address on each GPU comes from
// hipGetSymbolAddress and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[CSPD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
bool g_tried[kMaxDevices] = {};
hipError_t g_rc[kMaxDevices] = {};

}  // namespace

// Called by cspd_plan with `device` current: resolves the device address of
// that GPU's copy of the array, once per device.
void noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_tried[device]) return;
    g_tried[device] = true;
    void *ptr = nullptr;
    g_rc[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_ptr[device] = g_rc[device] == hipSuccess ? ptr : nullptr;
}

}  // namespace cspd

using namespace cspd;

extern "C" cspd_status cspd_omp_cross_scale_noalloc(cspd_plan_t p, int64_t B, const void *y, const uint8_t *mask,
                                                    const int32_t *k_scale, const int32_t *k_fine,
                                                    int32_t k_fine_uniform, int32_t *support, void *coef,
                                                    int32_t *k_used, void *xhat, int32_t *support_coarse,
                                                    void *hip_stream)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!p) return set_error(CSPD_E_INVALID, "plan is NULL");
        // profiling events are created per launch; this entry point records none
        ProfileSuspend quiet;
        // one scale: the full-dictionary kernels use no workspace
        if (p->s == 1)
            return cspd_omp_full(p, B, y, mask, k_fine, k_fine_uniform, support, coef, k_used, xhat, hip_stream);
        if (B < 0) return set_error(CSPD_E_INVALID, "B = %lld", (long long)B);
        if (!k_scale) return set_error(CSPD_E_INVALID, "k_scale is NULL");
        for (int s = 0; s + 1 < p->s; ++s)
            if (k_scale[s] < 0 || k_scale[s] > p->k_max)
                return set_error(CSPD_E_SHAPE, "k_scale[%d] = %d outside [0, k_max = %d]", s, k_scale[s], p->k_max);
        const size_t need = cross_call_workspace(p, B, k_scale, support_coarse != nullptr);
        if (need > (size_t)CSPD_NOALLOC_SCRATCH_BYTES)
            return set_error(CSPD_E_CAPACITY,
                             "%lld patches need %zu bytes of workspace; the static scratch holds %zu "
                             "(pass support_coarse, or split the batch)",
                             (long long)B, need, (size_t)CSPD_NOALLOC_SCRATCH_BYTES);
        if (p->device < 0 || p->device >= kMaxDevices)
            return set_error(CSPD_E_UNSUPPORTED, "device %d: the scratch table holds %d devices", p->device, kMaxDevices);
        void *work = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            if (!g_ptr[p->device])
                return set_error(CSPD_E_DEVICE, "device %d: address of the static scratch unavailable (%s)", p->device,
                                 g_tried[p->device] ? hipGetErrorString(g_rc[p->device]) : "never resolved");
            work = g_ptr[p->device];
        }
        return cross_scale_on(p, B, y, mask, k_scale, k_fine, k_fine_uniform, support, coef, k_used, xhat,
                              support_coarse, work, (size_t)CSPD_NOALLOC_SCRATCH_BYTES, (hipStream_t)hip_stream);
    });
}
