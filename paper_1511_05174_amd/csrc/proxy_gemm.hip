// First-scale correlations of a shared effective dictionary on the matrix
// cores: H = Y A_0 for a batch, i.e. h[b][i] = <a_i, y_b> for every patch b and
// every atom i of scale 0 (problem (P_low) of Section III-C under a dense
// measurement operator, where A_0 = Phi U D_0 is the same for all patches).
//
// This is the first proxy of Algorithm 1 (step 1, r = y) for all patches at
// once: a dense contraction over the measurement dimension, so it runs as a
// GEMM on the 32 x 32 x 2 FP32 MFMA.  The per-patch OMP then continues in
// candidate coordinates from H and the plan's Gram matrix and norms, without
// reading A_0 again.
//
// Layout: a wavefront owns 32 patches and walks the atoms in blocks of 32.
// MFMA operand A is the patch tile (lane l: patch l % 32), operand B the atom
// block (lane l: atom l % 32); the two k rows of each step split the
// coordinates in halves (lane l holds coordinates [(l / 32) LH, (l / 32 + 1)
// LH) of its patch and its atom).  The accumulator leaves lane l with atom
// l % 32 of patches 8 (r / 4) + 4 (l / 32) + r % 4, so each store instruction
// writes two 128-byte row segments of H.
#include <hip/hip_runtime.h>

#include "cspd_internal.h"

namespace cspd {
namespace gemm_impl {

constexpr int W = 4;   // wavefronts per workgroup

template <int LP>
__global__ __launch_bounds__(64 * W)
void k_proxy_gemm(const float *__restrict__ y, int y_stride, int m, int64_t nb, const float *__restrict__ v,
                  int lp, int t, float *__restrict__ h)
{
    constexpr int LH = LP / 2;
    typedef float acc_t __attribute__((ext_vector_type(16)));
    const int lane = threadIdx.x & 63;
    const int hh = lane >> 5;
    const int col = lane & 31;
    const int64_t p0 = ((int64_t)blockIdx.x * W + (threadIdx.x >> 6)) * 32;
    if (p0 >= nb) return;   // the whole wavefront leaves together
    // patch tile: lane holds patch p0 + col, coordinates [hh LH, hh LH + LH)
    // (rows past the batch and coordinates past m read a valid element and
    // are zeroed; nothing is stored for such rows)
    const int64_t prow = p0 + col < nb ? p0 + col : nb - 1;
    const float *yr = y + prow * (int64_t)y_stride;
    float ya[LH];
#pragma unroll
    for (int j = 0; j < LH; ++j) {
        const int c = hh * LH + j;
        const float val = yr[c < m ? c : 0];
        ya[j] = c < m ? val : 0.f;
    }
    for (int a0 = 0; a0 < t; a0 += 32) {
        // atom block: lane holds atom a0 + col (rows of v are zero past l)
        const int at = a0 + col < t ? a0 + col : t - 1;
        const float *vr = v + (int64_t)at * lp + hh * LH;
        float vb[LH];
#pragma unroll
        for (int j = 0; j < LH; j += 4) {
            const float4 q = *reinterpret_cast<const float4 *>(vr + j);
            vb[j] = q.x; vb[j + 1] = q.y; vb[j + 2] = q.z; vb[j + 3] = q.w;
        }
        acc_t acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
        for (int j = 0; j < LH; ++j) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ya[j], vb[j], acc, 0, 0, 0);
        if (a0 + col < t) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t p = p0 + 8 * (r >> 2) + 4 * hh + (r & 3);
                if (p < nb) h[p * t + a0 + col] = acc[r];
            }
        }
    }
}

template <int LP>
cspd_status launch(const ScaleArgs &a, float *h, hipStream_t st)
{
    const int64_t waves = (a.b + 31) / 32;
    const unsigned grid = (unsigned)((waves + W - 1) / W);
    launch_timed("proxy_gemm<f32>:s0", k_proxy_gemm<LP>, dim3(grid), dim3(64 * W), 0u, st, (const float *)a.y,
                 a.y_stride, a.m_dense, a.b, (const float *)a.v, a.lp, a.t, h);
    return hipGetLastError() == hipSuccess ? CSPD_OK : CSPD_E_DEVICE;
}

}  // namespace gemm_impl

bool proxy_gemm_fits(int dtype, const ScaleArgs &a)
{
    return dtype == CSPD_F32 && a.first && a.fold == kDense && a.lp >= 16 && a.lp <= 128 && a.l <= a.lp &&
           a.t >= 1 && a.m_dense == a.l;
}

cspd_status launch_proxy_gemm(int dtype, const ScaleArgs &a, float *h, hipStream_t st)
{
    if (!proxy_gemm_fits(dtype, a)) return CSPD_E_UNSUPPORTED;
    if (a.b <= 0) return CSPD_OK;
    switch (a.lp) {
        case 16: return gemm_impl::launch<16>(a, h, st);
        case 32: return gemm_impl::launch<32>(a, h, st);
        case 64: return gemm_impl::launch<64>(a, h, st);
        case 128: return gemm_impl::launch<128>(a, h, st);
        default: return CSPD_E_UNSUPPORTED;
    }
}

}  // namespace cspd
