// Whole-signal patch processing around the OMP calls (Section IV): cut a
// signal of up to 4 axes into overlapping patches (with their masks), and
// put patch estimates back together as the mean of every estimate that
// covers a sample.
//
// Grid: along each axis the patches start at 0, s, 2s, ... and, when the
// last regular start does not reach the end, once more at (dim - patch).
// Patches are numbered row-major over the grid; a patch is vectorised
// row-major over its own axes.
//
// Both kernels are plain HBM-bound gathers (no atomics, deterministic):
// extraction has one thread per patch sample (consecutive threads write
// consecutive samples of a patch); aggregation one thread per signal sample,
// which visits the covering patches in grid order and divides by their count.
#include <hip/hip_runtime.h>

#include "cspd_internal.h"

namespace cspd {
namespace patch_impl {

constexpr int AX = 4;   // axes handled by the kernels (leading axes padded with size 1)

struct Grid {
    int dims[AX];     // signal size per axis
    int patch[AX];    // patch size per axis
    int stride[AX];   // step per axis
    int reg[AX];      // regular positions per axis (0, s, ..., <= dim - patch)
    int cnt[AX];      // positions per axis (reg, plus the edge-aligned one when needed)
    int64_t sstride[AX];   // signal element stride per axis (row-major)
    int pvol;         // samples per patch
    int64_t npatch;   // patches
    int64_t nsig;     // signal samples
};

__device__ __forceinline__ int pos_of(const Grid &g, int d, int i)
{
    return i < g.reg[d] ? i * g.stride[d] : g.dims[d] - g.patch[d];
}

__global__ void k_extract(Grid g, const float *__restrict__ sig, const uint8_t *__restrict__ mask,
                          float *__restrict__ y, uint8_t *__restrict__ pmask)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.npatch * g.pvol) return;
    const int64_t b = t / g.pvol;
    int e = (int)(t - b * g.pvol);
    int64_t pb = b;
    int64_t off = 0;
    // last axis fastest, for both the grid index and the in-patch index
#pragma unroll
    for (int d = AX - 1; d >= 0; --d) {
        const int gi = (int)(pb % g.cnt[d]);
        pb /= g.cnt[d];
        const int ei = e % g.patch[d];
        e /= g.patch[d];
        off += (int64_t)(pos_of(g, d, gi) + ei) * g.sstride[d];
    }
    y[t] = sig[off];
    if (pmask) pmask[t] = mask ? mask[off] : (uint8_t)1;
}

__global__ void k_aggregate(Grid g, const float *__restrict__ est, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.nsig) return;
    int x[AX];
    int64_t r = t;
#pragma unroll
    for (int d = AX - 1; d >= 0; --d) {
        x[d] = (int)(r % g.dims[d]);
        r /= g.dims[d];
    }
    // covering grid indices per axis: the regular ones lo .. lo + nr - 1,
    // then the edge-aligned one (index reg) when it exists and covers x
    int lo[AX], nc[AX], nr[AX];
#pragma unroll
    for (int d = 0; d < AX; ++d) {
        const int p = g.patch[d], s = g.stride[d];
        const int a = x[d] - p + 1;
        const int l = a <= 0 ? 0 : (a + s - 1) / s;
        int h = x[d] / s;
        if (h > g.reg[d] - 1) h = g.reg[d] - 1;
        lo[d] = l;
        nr[d] = h >= l ? h - l + 1 : 0;
        nc[d] = nr[d] + ((g.cnt[d] > g.reg[d] && x[d] >= g.dims[d] - p) ? 1 : 0);
    }
    double acc = 0.0;
    int n = 0;
    // grid order (first axis slowest), as the patches are numbered
    for (int j0 = 0; j0 < nc[0]; ++j0) {
        const int g0 = j0 < nr[0] ? lo[0] + j0 : g.reg[0];
        for (int j1 = 0; j1 < nc[1]; ++j1) {
            const int g1 = j1 < nr[1] ? lo[1] + j1 : g.reg[1];
            for (int j2 = 0; j2 < nc[2]; ++j2) {
                const int g2 = j2 < nr[2] ? lo[2] + j2 : g.reg[2];
                for (int j3 = 0; j3 < nc[3]; ++j3) {
                    const int g3 = j3 < nr[3] ? lo[3] + j3 : g.reg[3];
                    const int gi[AX] = {g0, g1, g2, g3};
                    int64_t b = 0;
                    int e = 0;
#pragma unroll
                    for (int d = 0; d < AX; ++d) {
                        b = b * g.cnt[d] + gi[d];
                        e = e * g.patch[d] + (x[d] - pos_of(g, d, gi[d]));
                    }
                    acc += (double)est[b * g.pvol + e];
                    ++n;
                }
            }
        }
    }
    out[t] = (float)(acc / (double)n);
}

}  // namespace patch_impl
}  // namespace cspd

using namespace cspd;
using namespace cspd::patch_impl;

namespace {

// Validates a grid description and fills the kernels' form of it.
cspd_status make_grid(const cspd_patch_grid *d, Grid &g)
{
    if (!d) return set_error(CSPD_E_INVALID, "grid is NULL");
    if (d->ndim < 1 || d->ndim > AX) return set_error(CSPD_E_INVALID, "ndim %d outside 1..%d", d->ndim, AX);
    const int lead = AX - d->ndim;
    int64_t nsig = 1, pvol = 1, np = 1;
    for (int k = 0; k < AX; ++k) {
        const int src = k - lead;
        const int dim = src >= 0 ? d->dims[src] : 1;
        const int p = src >= 0 ? d->patch[src] : 1;
        const int s = src >= 0 ? d->stride[src] : 1;
        if (dim < 1 || p < 1 || p > dim || s < 1)
            return set_error(CSPD_E_SHAPE, "axis %d: dim %d patch %d stride %d", src, dim, p, s);
        g.dims[k] = dim;
        g.patch[k] = p;
        g.stride[k] = s;
        g.reg[k] = (dim - p) / s + 1;
        g.cnt[k] = g.reg[k] + ((dim - p) % s != 0 ? 1 : 0);
        nsig *= dim;
        pvol *= p;
        np *= g.cnt[k];
    }
    int64_t st = 1;
    for (int k = AX - 1; k >= 0; --k) {
        g.sstride[k] = st;
        st *= g.dims[k];
    }
    if (pvol > 65536) return set_error(CSPD_E_SHAPE, "patch volume %lld above 65536", (long long)pvol);
    if (nsig >= ((int64_t)1 << 38) || np * pvol >= ((int64_t)1 << 38))
        return set_error(CSPD_E_SHAPE, "signal too large");
    g.pvol = (int)pvol;
    g.npatch = np;
    g.nsig = nsig;
    return CSPD_OK;
}

}  // namespace

extern "C" {

int64_t cspd_patch_count(const cspd_patch_grid *grid)
{
    clear_error();
    Grid g{};
    if (make_grid(grid, g) != CSPD_OK) return -1;
    return g.npatch;
}

cspd_status cspd_extract_patches(const cspd_patch_grid *grid, const float *signal, const uint8_t *mask, float *y,
                                 uint8_t *patch_mask, void *hip_stream)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        Grid g{};
        cspd_status rc = make_grid(grid, g);
        if (rc != CSPD_OK) return rc;
        if (!signal || !y) return set_error(CSPD_E_INVALID, "signal / y is NULL");
        const int64_t n = g.npatch * g.pvol;
        const int bs = 256;
        ProfileToken *tok = profile_begin("extract_patches", (hipStream_t)hip_stream);
        hipLaunchKernelGGL(k_extract, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, (hipStream_t)hip_stream, g,
                           signal, mask, y, patch_mask);
        profile_end(tok, (hipStream_t)hip_stream);
        if (hipGetLastError() != hipSuccess) return set_error(CSPD_E_DEVICE, "extract launch failed");
        return CSPD_OK;
    });
}

cspd_status cspd_aggregate_patches(const cspd_patch_grid *grid, const float *estimates, float *signal_out,
                                   void *hip_stream)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        Grid g{};
        cspd_status rc = make_grid(grid, g);
        if (rc != CSPD_OK) return rc;
        if (!estimates || !signal_out) return set_error(CSPD_E_INVALID, "estimates / signal_out is NULL");
        const int bs = 256;
        ProfileToken *tok = profile_begin("aggregate_patches", (hipStream_t)hip_stream);
        hipLaunchKernelGGL(k_aggregate, dim3((unsigned)((g.nsig + bs - 1) / bs)), dim3(bs), 0, (hipStream_t)hip_stream,
                           g, estimates, signal_out);
        profile_end(tok, (hipStream_t)hip_stream);
        if (hipGetLastError() != hipSuccess) return set_error(CSPD_E_DEVICE, "aggregate launch failed");
        return CSPD_OK;
    });
}

}  // extern "C"
