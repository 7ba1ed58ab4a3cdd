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
//
// Reduced-precision variant (a precision option, not in the paper): the same
// tiles on the bf16 / fp16 matrix cores (v_mfma_f32_32x32x16_*, FP32
// accumulation) from the plan's 16-bit copy of A_0 and a 16-bit copy of each
// patch scaled by a power of two to a largest entry in [0.5, 1) (the scale is
// undone exactly on the accumulators).  Lane half h supplies coordinates
// h LH + 8 g + [0, 8) at step g on both operands.  The per-patch OMP then
// re-scores its candidates in FP32 before each pick.
#include <hip/hip_runtime.h>

#include <climits>

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

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int LP, bool BF16>
__global__ __launch_bounds__(64 * W)
void k_proxy_gemm_lo(const float *__restrict__ y, int y_stride, int m, int64_t nb,
                     const uint16_t *__restrict__ vlo, int lp, int t, float *__restrict__ h)
{
    constexpr int LH = LP / 2;
    constexpr int NG = LH / 8;
    static_assert(NG >= 1 && LH % 8 == 0, "8 coordinates per lane and step");
    typedef float acc_t __attribute__((ext_vector_type(16)));
    const int lane = threadIdx.x & 63;
    const int hh = lane >> 5;
    const int col = lane & 31;
    const int64_t p0 = ((int64_t)blockIdx.x * W + (threadIdx.x >> 6)) * 32;
    if (p0 >= nb) return;   // the whole wavefront leaves together
    const int64_t prow = p0 + col < nb ? p0 + col : nb - 1;
    const float *yr = y + prow * (int64_t)y_stride;
    float ya[LH];
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < LH; ++j) {
        const int c = hh * LH + j;
        const float val = yr[c < m ? c : 0];
        ya[j] = c < m ? val : 0.f;
        mx = fmaxf(mx, fabsf(ya[j]));
    }
    {
        // lanes l and l + 32 hold the two halves of the same patch
        auto rs = __builtin_amdgcn_permlane32_swap(__float_as_int(mx), __float_as_int(mx), false, false);
        mx = fmaxf(__int_as_float(rs[0]), __int_as_float(rs[1]));
    }
    int ex = 0;
    (void)frexpf(mx, &ex);                   // mx = f 2^ex, f in [0.5, 1)
    ex = ex < -100 ? -100 : (ex > 100 ? 100 : ex);
    const float sc = mx > 0.f ? ldexpf(1.f, -ex) : 1.f;
    const float inv = mx > 0.f ? ldexpf(1.f, ex) : 1.f;
    unsigned yl[NG][4];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float f0 = ya[8 * g + 2 * i] * sc, f1 = ya[8 * g + 2 * i + 1] * sc;
            unsigned lo, hi;
            if constexpr (BF16) {
                unsigned u0 = __float_as_uint(f0), u1 = __float_as_uint(f1);
                u0 += 0x7fffu + ((u0 >> 16) & 1u);   // round to nearest even
                u1 += 0x7fffu + ((u1 >> 16) & 1u);
                lo = u0 >> 16;
                hi = u1 >> 16;
            } else {
                const _Float16 a0 = (_Float16)f0, a1 = (_Float16)f1;
                lo = *reinterpret_cast<const unsigned short *>(&a0);
                hi = *reinterpret_cast<const unsigned short *>(&a1);
            }
            yl[g][i] = lo | (hi << 16);
        }
    }
    // inverse scale of the patch row each accumulator entry belongs to
    float rinv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) rinv[r] = __shfl(inv, 8 * (r >> 2) + 4 * hh + (r & 3), 64);
    for (int a0 = 0; a0 < t; a0 += 32) {
        const int at = a0 + col < t ? a0 + col : t - 1;
        const uint16_t *vr = vlo + (int64_t)at * lp + hh * LH;
        acc_t acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const uint4 q = *reinterpret_cast<const uint4 *>(vr + 8 * g);
            const unsigned xb[4] = {q.x, q.y, q.z, q.w};
            if constexpr (BF16) {
                bf16x8 xa, xv;
                __builtin_memcpy(&xa, yl[g], 16);
                __builtin_memcpy(&xv, xb, 16);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, xv, acc, 0, 0, 0);
            } else {
                f16x8 xa, xv;
                __builtin_memcpy(&xa, yl[g], 16);
                __builtin_memcpy(&xv, xb, 16);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(xa, xv, acc, 0, 0, 0);
            }
        }
        if (a0 + col < t) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t p = p0 + 8 * (r >> 2) + 4 * hh + (r & 3);
                if (p < nb) h[p * t + a0 + col] = acc[r] * rinv[r];
            }
        }
    }
}

// ---- plans with several operators: the batch grouped by operator ----------
// Each patch's first-scale correlations use its own operator's A_0, so the
// patches are listed operator by operator (a counting sort of the patch
// indices) and each wavefront takes up to 32 patches of one operator.  The
// order of the patches within an operator does not matter: every output is
// one dot product, summed in the same order whatever the tile holds.
// Patches whose operator is out of range are left out (they stay unsolved).
// One workgroup lists the whole batch: operator counts in LDS, their prefix
// sums (first position and first tile of each operator), then each patch
// index written at its operator's next position (LDS cursors).  One launch,
// no global counters to clear; the batch is read twice, 1,024 patches a step.
constexpr int kMaxGroups = 4096;   // operators per plan
constexpr int kGroupThreads = 1024;

__global__ __launch_bounds__(kGroupThreads) void k_groups(const int *__restrict__ phase, int64_t nb, int P,
                                                          int *__restrict__ seg, int *__restrict__ tile,
                                                          int *__restrict__ perm)
{
    __shared__ int cnt[kMaxGroups];
    __shared__ int cur[kMaxGroups];
    for (int i = threadIdx.x; i < P; i += kGroupThreads) cnt[i] = 0;
    __syncthreads();
    for (int64_t b = threadIdx.x; b < nb; b += kGroupThreads) {
        const int ph = phase[b];
        if (ph >= 0 && ph < P) atomicAdd(&cnt[ph], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0, t = 0;
        for (int i = 0; i < P; ++i) {
            seg[i] = s;
            tile[i] = t;
            cur[i] = s;
            s += cnt[i];
            t += (cnt[i] + 31) / 32;
        }
        seg[P] = s;
        tile[P] = t;
    }
    __syncthreads();
    for (int64_t b = threadIdx.x; b < nb; b += kGroupThreads) {
        const int ph = phase[b];
        if (ph >= 0 && ph < P) perm[atomicAdd(&cur[ph], 1)] = (int)b;
    }
}

// k_proxy_gemm over the grouped batch: wavefront w takes tile w (32 patches
// of one operator, the last tile of an operator ragged)
template <int LP>
__global__ __launch_bounds__(64 * W)
void k_proxy_gemm_groups(const float *__restrict__ y, int y_stride, int m, const float *__restrict__ v, int lp,
                         int t, int64_t phase_stride, int P, const int *__restrict__ seg,
                         const int *__restrict__ tile, const int *__restrict__ perm, float *__restrict__ h)
{
    constexpr int LH = LP / 2;
    typedef float acc_t __attribute__((ext_vector_type(16)));
    const int lane = threadIdx.x & 63;
    const int hh = lane >> 5;
    const int col = lane & 31;
    const int w = blockIdx.x * W + (threadIdx.x >> 6);
    if (w >= tile[P]) return;   // the whole wavefront leaves together
    // operator of tile w: the largest ph with tile[ph] <= w (empty operators
    // share their bound with the next one)
    int lo = 0, hi = P;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile[mid] <= w) lo = mid;
        else hi = mid;
    }
    const int ph = lo;
    const int first = seg[ph] + (w - tile[ph]) * 32;
    const int nrow = seg[ph + 1] - first < 32 ? seg[ph + 1] - first : 32;
    const int64_t prow = perm[first + (col < nrow ? col : 0)];
    const float *yr = y + prow * (int64_t)y_stride;
    float ya[LH];
#pragma unroll
    for (int j = 0; j < LH; ++j) {
        const int c = hh * LH + j;
        const float val = yr[c < m ? c : 0];
        ya[j] = (c < m && col < nrow) ? val : 0.f;
    }
    const float *vph = v + (int64_t)ph * phase_stride;
    for (int a0 = 0; a0 < t; a0 += 32) {
        const int at = a0 + col < t ? a0 + col : t - 1;
        const float *vr = vph + (int64_t)at * lp + hh * LH;
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
                const int rr = 8 * (r >> 2) + 4 * hh + (r & 3);
                if (rr < nrow) h[(int64_t)perm[first + rr] * t + a0 + col] = acc[r];
            }
        }
    }
}

template <int LP>
cspd_status launch_groups(const ScaleArgs &a, float *h, hipStream_t st)
{
    const int P = a.n_phases;
    if (a.b >= (int64_t)INT_MAX || P > kMaxGroups) return CSPD_E_UNSUPPORTED;   // patch indices are 32-bit
    const PhaseGroups g = phase_groups((char *)h + phase_groups_offset(a.b, a.t), a.b, P);
    hipLaunchKernelGGL(k_groups, dim3(1), dim3(kGroupThreads), 0, st, a.phase, a.b, P, g.seg, g.tile, g.perm);
    // at most ceil(B / 32) full tiles plus one ragged tile per operator
    const int64_t waves = (a.b + 31) / 32 + P;
    const unsigned grid = (unsigned)((waves + W - 1) / W);
    launch_timed("proxy_gemm<f32,groups>:s0", k_proxy_gemm_groups<LP>, dim3(grid), dim3(64 * W), 0u, st,
                 (const float *)a.y, a.y_stride, a.m_dense, (const float *)a.v, a.lp, a.t, a.phase_stride, P,
                 (const int *)g.seg, (const int *)g.tile, (const int *)g.perm, h);
    return hipGetLastError() == hipSuccess ? CSPD_OK : CSPD_E_DEVICE;
}

template <int LP>
cspd_status launch(const ScaleArgs &a, float *h, hipStream_t st)
{
    if (a.phase && a.n_phases > 1) return launch_groups<LP>(a, h, st);
    const int64_t waves = (a.b + 31) / 32;
    const unsigned grid = (unsigned)((waves + W - 1) / W);
    if (a.hre > 0 && a.vlo) {
        if (a.corr_lo == CSPD_CORR_BF16_RESCORE)
            launch_timed("proxy_gemm<bf16>:s0", k_proxy_gemm_lo<LP, true>, dim3(grid), dim3(64 * W), 0u, st,
                         (const float *)a.y, a.y_stride, a.m_dense, a.b, (const uint16_t *)a.vlo, a.lp, a.t, h);
        else
            launch_timed("proxy_gemm<f16>:s0", k_proxy_gemm_lo<LP, false>, dim3(grid), dim3(64 * W), 0u, st,
                         (const float *)a.y, a.y_stride, a.m_dense, a.b, (const uint16_t *)a.vlo, a.lp, a.t, h);
        return hipGetLastError() == hipSuccess ? CSPD_OK : CSPD_E_DEVICE;
    }
    launch_timed("proxy_gemm<f32>:s0", k_proxy_gemm<LP>, dim3(grid), dim3(64 * W), 0u, st, (const float *)a.y,
                 a.y_stride, a.m_dense, a.b, (const float *)a.v, a.lp, a.t, h);
    return hipGetLastError() == hipSuccess ? CSPD_OK : CSPD_E_DEVICE;
}

}  // namespace gemm_impl

size_t phase_groups_offset(int64_t B, int t)
{
    return ((size_t)B * (size_t)t * sizeof(float) + 255) / 256 * 256;
}

size_t phase_groups_bytes(int64_t B, int P)
{
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    return 2 * al(sizeof(int) * (size_t)(P + 1)) + al(sizeof(int) * (size_t)B);
}

PhaseGroups phase_groups(void *base, int64_t B, int P)
{
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    char *c = (char *)base;
    PhaseGroups g;
    g.seg = (int *)c;
    c += al(sizeof(int) * (size_t)(P + 1));
    g.tile = (int *)c;
    c += al(sizeof(int) * (size_t)(P + 1));
    g.perm = (int *)c;
    return g;
}

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
