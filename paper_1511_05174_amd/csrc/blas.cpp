// Plain library GEMMs (rocBLAS) for the full-search path over large shared
// dictionaries: the plan's Gram matrix A^T A and each call's correlations
// A^T Y.  One rocBLAS handle per device, created on first use; a call binds
// it to the caller's stream under a lock, so calls from several threads do
// not race on the handle's stream.
#include <rocblas/rocblas.h>

#include <mutex>

#include "cspd_internal.h"

namespace cspd {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
rocblas_handle g_handle[kMaxDevices] = {};

}  // namespace

cspd_status gemm_tn_f64(int device, hipStream_t st, int m, int n, int k, const double *a, int lda,
                        const double *b, int ldb, double *c, int ldc)
{
    if (device < 0 || device >= kMaxDevices) return set_error(CSPD_E_DEVICE, "device %d out of range", device);
    if (m <= 0 || n <= 0) return CSPD_OK;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_handle[device] && rocblas_create_handle(&g_handle[device]) != rocblas_status_success) {
        g_handle[device] = nullptr;
        return set_error(CSPD_E_DEVICE, "rocblas_create_handle failed on device %d", device);
    }
    rocblas_handle h = g_handle[device];
    if (rocblas_set_stream(h, st) != rocblas_status_success)
        return set_error(CSPD_E_DEVICE, "rocblas_set_stream failed");
    const double one = 1.0, zero = 0.0;
    // column-major: C (m x n) = A^T B, A stored k x m, B stored k x n
    const rocblas_status rs = rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, m, n, k, &one,
                                            a, lda, b, ldb, &zero, c, ldc);
    if (rs != rocblas_status_success) return set_error(CSPD_E_DEVICE, "rocblas_dgemm failed (status %d)", (int)rs);
    return CSPD_OK;
}

}  // namespace cspd
