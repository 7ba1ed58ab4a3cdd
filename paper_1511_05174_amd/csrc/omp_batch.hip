// Full-dictionary OMP (Algorithm 1) over a large shared dictionary in
// coefficient coordinates, for dictionaries beyond the per-patch kernels
// (up to 8192 atoms of any length, sparsity up to 64): the work of the
// paper's single-scale comparators (Section II-C and Section IV's time versus
// accuracy study).
//
// With A the shared effective dictionary (Phi D, or D under the identity),
// G = A^T A is formed once per plan and p0 = A^T y once per call for the
// whole batch (plain library GEMMs, FP64).  Algorithm 1 then needs neither
// y nor A again: after the support Omega has reached k atoms with
// coefficients alpha (least squares on A_Omega), the proxy is
//     c = A^T (y - A_Omega alpha) = p0 - G[:, Omega] alpha,
// the support merge and projection grow an FP64 Cholesky factor of
// G[Omega, Omega] by one row per step (w = L^{-1} G[Omega, k], pivot
// G[k, k] - |w|^2, z_k = (p0_k - w^T z) / pivot^(1/2)), and alpha = L^{-T} z.
// The proxy reads G stored in FP32 (its rounding, about 1e-7 of the
// correlations, stays far below the near-tie level); the Cholesky factor
// takes its entries <a_k, a_j> exactly, as FP64 dot products of the stored
// FP64 atoms, so the coefficients keep FP64 accuracy on ill-conditioned
// supports.
//
// One workgroup (four wavefronts) per patch: thread t owns atoms t, t + 256,
// ... of the proxy, held in FP64 registers (p0 and G[:, Omega] alpha); each
// step reads the k + 1 rows of G of the support (G is symmetric, so rows
// are columns) with coalesced loads.  The argmax takes the lowest atom index
// on ties.
//
// The same kernel runs the finest scale of zero-tree OMP (Algorithm 2) when
// its vectors are long: the candidates are then the children of the coarse
// support (candidate c is child c mod Q of the (c / Q)-th coarse atom), their
// correlations <a_i, y> are formed in the kernel (FP64 sums of the FP32
// vectors, one wavefront per candidate), and the proxy gathers G[Omega, i]
// over the candidates only.  Wavefront 0 runs the triangular solves column by column, lane j
// holding row j.  An atom whose squared pivot is at most 1e-10 of its squared
// norm is dependent and ends the patch, as does reaching the rank of the
// measurement space.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>

#include "cspd_internal.h"

namespace cspd {
namespace batch_impl {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

struct BatchArgs {
    int64_t b;
    const double *p0;      // b x t: <a_i, y_b>
    const float *g;        // t x t Gram matrix of the effective atoms (FP32)
    const double *a64;     // t x l effective atoms (FP64)
    int l;
    int t;
    int rank;              // rank bound of the measurement space
    const int *kvec;       // b or null
    int kuni;
    int kcap;              // row stride of support / coef and cap of k
    int *support;
    float *coef;
    int *k_used;
    float *xhat;           // b x n or null
    const float *dh;       // t x n atoms in signal coordinates
    int n;
    // candidate mode (zero-tree finest scale): children of the coarse support
    const float *y;        // b x y_stride measurements
    int y_stride;
    const float *v;        // t x lp effective atoms (FP32)
    int lp;
    const int *prev_sup;   // b x prev_stride coarse supports
    int prev_stride;
    const int *prev_kused; // b
    int q;                 // children per coarse atom
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double shfl_d(double v, int src)
{
    const int lo = __shfl(__double2loint(v), src, 64);
    const int hi = __shfl(__double2hiint(v), src, 64);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double shfl_xor_d(double v, int m)
{
    const int lo = __shfl_xor(__double2loint(v), m, 64);
    const int hi = __shfl_xor(__double2hiint(v), m, 64);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
    return v;
}

template <int TPT, int KX, bool CAND>
__global__ __launch_bounds__(kThreads) void k_omp_batch(BatchArgs a)
{
    static_assert(TPT >= 1 && TPT <= 32 && KX <= 64, "atoms per thread, sparsity");
    constexpr int NCX = CAND ? TPT * kThreads : 1;
    __shared__ double sp0[NCX];      // candidate mode: <a_i, y> of every candidate
    __shared__ double sL[KX * KX];
    __shared__ double sz[KX], sal[KX], sg[KX + 1];
    __shared__ int ssup[KX];
    __shared__ double wbs[kWaves];
    __shared__ int wbi[kWaves];
    __shared__ int s_pick, s_go;
    __shared__ double s_p0k;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int64_t b = blockIdx.x;
    const int t = a.t;
    const double *p0 = CAND ? nullptr : a.p0 + b * (int64_t)t;

    // candidates: every atom, or the children of the coarse support
    int nc = t;
    if constexpr (CAND) {
        const int kp = a.prev_kused[b];
        nc = kp * a.q;
        nc = nc < NCX ? nc : NCX;
    }
    auto atom_of = [&](int ci) -> int {
        if constexpr (!CAND) return ci;
        const int pj = ci / a.q;
        return a.prev_sup[b * (int64_t)a.prev_stride + pj] * a.q + (ci - pj * a.q);
    };
    if constexpr (CAND) {
        // <a_i, y> of each candidate: one wavefront per candidate, FP64 sums
        const float *yr = a.y + b * (int64_t)a.y_stride;
        for (int ci = wv; ci < nc; ci += kWaves) {
            const float *vr = a.v + (int64_t)atom_of(ci) * a.lp;
            double part = 0.0;
            for (int c = lane; c < a.l; c += 64) part += (double)vr[c] * (double)yr[c];
            part = wave_sum_d(part);
            if (lane == 0) sp0[ci] = part;
        }
        __syncthreads();
    }
    double pr[TPT], beta[TPT];
    double inv[TPT];
    int at[TPT];
    unsigned sel = 0u;
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        const int ci = tid + q * kThreads;
        const bool live = ci < nc;
        at[q] = live ? atom_of(ci) : INT_MAX;
        pr[q] = live ? (CAND ? sp0[ci] : p0[ci]) : 0.0;
        beta[q] = 0.0;
        const double gii = live ? (double)a.g[(int64_t)at[q] * t + at[q]] : 0.0;
        inv[q] = gii > 0.0 ? 1.0 / sqrt(gii) : -1.0;   // an effective column of zero is never picked
    }
    int K = a.kvec ? a.kvec[b] : a.kuni;
    K = K < a.kcap ? K : a.kcap;
    K = K < KX ? K : KX;
    K = K < nc ? K : nc;
    K = K > 0 ? K : 0;

    int nsel = 0;
    for (int it = 0; it < K; ++it) {
        // ---- proxy and argmax: |p0 - G[:, Omega] alpha| / ||a_i||
        double bs = -1.0;
        int bi = INT_MAX;
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
            const bool ok = at[q] != INT_MAX && inv[q] > 0.0 && !((sel >> q) & 1u);
            const double sc = ok ? fabs(pr[q] - beta[q]) * inv[q] : -1.0;
            if (sc > bs || (sc == bs && at[q] < bi)) { bs = sc; bi = at[q]; }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            const double os = shfl_xor_d(bs, m);
            const int oi = __shfl_xor(bi, m, 64);
            if (os > bs || (os == bs && oi < bi)) { bs = os; bi = oi; }
        }
        if (lane == 0) { wbs[wv] = bs; wbi[wv] = bi; }
        __syncthreads();
        if (tid == 0) {
            double best = wbs[0];
            int bidx = wbi[0];
            for (int w = 1; w < kWaves; ++w)
                if (wbs[w] > best || (wbs[w] == best && wbi[w] < bidx)) { best = wbs[w]; bidx = wbi[w]; }
            s_pick = best >= 0.0 ? bidx : -1;
        }
        __syncthreads();
        const int k = s_pick;
        if (k < 0) break;                    // no candidate left
#pragma unroll
        for (int q = 0; q < TPT; ++q)
            if (at[q] == k) s_p0k = pr[q];   // <a_k, y>, from the thread that holds it
        // ---- support merge: Gram entries of the new atom against Omega and
        // its squared norm (entry it), FP64 dot products, one per wavefront
        {
            const double *ak = a.a64 + (int64_t)k * a.l;
            for (int j = wv; j <= it; j += kWaves) {
                const double *aj = j < it ? a.a64 + (int64_t)ssup[j] * a.l : ak;
                double part = 0.0;
                for (int c = lane; c < a.l; c += 64) part += ak[c] * aj[c];
                part = wave_sum_d(part);
                if (lane == 0) sg[j] = part;
            }
        }
        __syncthreads();
        if (wv == 0) {
            // w = L^{-1} g, column by column (lane j holds row j)
            double gj = lane < it ? sg[lane] : 0.0;
            double wj = 0.0;
            for (int i = 0; i < it; ++i) {
                const double wi = shfl_d(gj, i) / sL[i * KX + i];
                if (lane == i) wj = wi;
                if (lane > i && lane < it) gj -= sL[lane * KX + i] * wi;
            }
            const double ww = wave_sum_d(lane < it ? wj * wj : 0.0);
            const double zw = wave_sum_d(lane < it ? wj * sz[lane] : 0.0);
            const double gkk = sg[it];
            const double piv = gkk - ww;
            const bool ok = piv > 1e-10 * gkk && it < a.rank;
            if (ok) {
                // ---- projection: new row of L, z_k, then alpha = L^{-T} z
                const double l = sqrt(piv);
                if (lane < it) sL[it * KX + lane] = wj;
                if (lane == 0) {
                    sL[it * KX + it] = l;
                    sz[it] = (s_p0k - zw) / l;
                    ssup[it] = k;
                }
                wave_sync();
                double zm = lane <= it ? sz[lane] : 0.0;
                double al = 0.0;
                for (int i = it; i >= 0; --i) {
                    const double ai = shfl_d(zm, i) / sL[i * KX + i];
                    if (lane == i) al = ai;
                    if (lane < i) zm -= sL[i * KX + lane] * ai;
                }
                if (lane <= it) sal[lane] = al;
            }
            if (lane == 0) s_go = ok ? 1 : 0;
        }
        __syncthreads();
        if (!s_go) break;                    // dependent atom, or the space is spanned
#pragma unroll
        for (int q = 0; q < TPT; ++q)
            if (at[q] == k) sel |= 1u << q;
        nsel = it + 1;
        // ---- residue in coefficient coordinates: G[:, Omega] alpha
#pragma unroll
        for (int q = 0; q < TPT; ++q) beta[q] = 0.0;
        for (int j = 0; j <= it; ++j) {
            const float *row = a.g + (int64_t)ssup[j] * t;
            const double aj = sal[j];
#pragma unroll
            for (int q = 0; q < TPT; ++q)
                if (at[q] != INT_MAX) beta[q] += (double)row[at[q]] * aj;
        }
    }

    // ---- outputs
    if (tid == 0) a.k_used[b] = nsel;
    for (int i = tid; i < a.kcap; i += kThreads) {
        a.support[b * (int64_t)a.kcap + i] = i < nsel ? ssup[i] : -1;
        a.coef[b * (int64_t)a.kcap + i] = i < nsel ? (float)sal[i] : 0.f;
    }
    if (a.xhat) {
        for (int c = tid; c < a.n; c += kThreads) {
            double acc = 0.0;
            for (int j = 0; j < nsel; ++j) acc += sal[j] * (double)a.dh[(int64_t)ssup[j] * a.n + c];
            a.xhat[b * (int64_t)a.n + c] = (float)acc;
        }
    }
}

// y (b x m, FP32, row stride ys) to FP64 (b x m).
__global__ void k_to_f64(const float *__restrict__ y, int ys, int m, int64_t nb, double *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nb * m) return;
    const int64_t r = idx / m;
    const int c = (int)(idx % m);
    out[idx] = (double)y[r * ys + c];
}

template <int TPT, int KX, bool CAND>
void launch_one(const BatchArgs &a, int scale, hipStream_t st)
{
    char label[64];
    if (CAND)
        snprintf(label, sizeof(label), "omp_batch<f32,c%d,k%d>:s%d", TPT * kThreads, KX, scale);
    else
        snprintf(label, sizeof(label), "omp_batch<f32,t%d,k%d>:full", TPT * kThreads, KX);
    launch_timed(label, k_omp_batch<TPT, KX, CAND>, dim3((unsigned)a.b), dim3(kThreads), 0u, st, a);
}

// n: atoms (full search) or the most candidates (zero-tree finest scale)
template <int KX, bool CAND>
cspd_status by_n(const BatchArgs &a, int n, int scale, hipStream_t st)
{
    if (CAND && n <= 256) launch_one<1, KX, CAND>(a, scale, st);
    else if (CAND && n <= 512) launch_one<2, KX, CAND>(a, scale, st);
    else if (n <= 1024) launch_one<4, KX, CAND>(a, scale, st);
    else if (n <= 2048) launch_one<8, KX, CAND>(a, scale, st);
    else if (n <= 4096) launch_one<16, KX, CAND>(a, scale, st);
    else if (n <= 8192) launch_one<32, KX, CAND>(a, scale, st);
    else return CSPD_E_UNSUPPORTED;
    return hipGetLastError() == hipSuccess ? CSPD_OK : CSPD_E_DEVICE;
}

}  // namespace batch_impl

bool batch_fits(const cspd_plan_s *p)
{
    const ScalePlan &sc = p->sc[p->s - 1];
    return p->bat_g != nullptr && p->bat_a64 != nullptr && sc.t <= kMaxBatchAtoms && p->n_phases == 1;
}

// Patches per chunk of a batch call: p0 and the FP64 copy of y of a chunk
// stay within about 1 GiB of stream-ordered workspace.
static int64_t batch_chunk(const cspd_plan_s *p)
{
    const ScalePlan &sc = p->sc[p->s - 1];
    const int64_t per = (int64_t)sizeof(double) * ((int64_t)sc.t + sc.l);
    int64_t c = ((int64_t)1 << 30) / per;
    c = c < 65536 ? c : 65536;
    return c > 256 ? c : 256;
}

cspd_status launch_batch(const cspd_plan_s *p, const ScaleArgs &a, int max_cand, hipStream_t st)
{
    using namespace batch_impl;
    if (!batch_fits(p) || max_cand > kMaxBatchAtoms) return CSPD_E_UNSUPPORTED;
    if (a.b <= 0) return CSPD_OK;
    const ScalePlan &sc = p->sc[p->s - 1];
    const int kmax = a.kvec ? p->k_max : a.kuni;
    if (!a.first) {
        // zero-tree finest scale: candidates = children of the coarse support
        BatchArgs ba{};
        ba.b = a.b;
        ba.g = (const float *)p->bat_g;
        ba.a64 = (const double *)p->bat_a64;
        ba.l = sc.l;
        ba.t = sc.t;
        ba.rank = a.fold == kDense ? a.m_dense : sc.l;
        ba.kvec = a.kvec;
        ba.kuni = a.kuni;
        ba.kcap = a.sup_count;
        ba.support = a.sup_out;
        ba.coef = (float *)a.coef_out;
        ba.k_used = a.kused_out;
        ba.xhat = (float *)a.xhat;
        ba.dh = (const float *)p->d_high;
        ba.n = a.n;
        ba.y = (const float *)a.y;
        ba.y_stride = a.y_stride;
        ba.v = (const float *)sc.v;
        ba.lp = sc.lp;
        ba.prev_sup = a.prev_sup;
        ba.prev_stride = a.prev_stride;
        ba.prev_kused = a.prev_kused;
        ba.q = a.q;
        const cspd_status rc = kmax <= 16 ? by_n<16, true>(ba, max_cand, a.scale, st)
                                          : by_n<64, true>(ba, max_cand, a.scale, st);
        if (rc != CSPD_OK && !has_error()) return set_error(rc, "zero-tree batch kernel launch failed");
        return rc;
    }
    const int64_t chunk = batch_chunk(p);
    const int64_t cb = a.b < chunk ? a.b : chunk;
    double *ws = nullptr;
    const size_t wbytes = sizeof(double) * (size_t)cb * ((size_t)sc.t + (size_t)sc.l);
    if (hipMallocAsync((void **)&ws, wbytes, st) != hipSuccess)
        return set_error(CSPD_E_NOMEM, "batch OMP workspace of %zu bytes", wbytes);
    double *p0 = ws;
    double *y64 = ws + (size_t)cb * sc.t;
    cspd_status rc = CSPD_OK;
    for (int64_t b0 = 0; b0 < a.b && rc == CSPD_OK; b0 += cb) {
        const int64_t nb = a.b - b0 < cb ? a.b - b0 : cb;
        const int64_t tot = nb * (int64_t)sc.l;
        k_to_f64<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>((const float *)a.y + b0 * a.y_stride, a.y_stride,
                                                                 sc.l, nb, y64);
        if (hipGetLastError() != hipSuccess) { rc = set_error(CSPD_E_DEVICE, "conversion kernel launch failed"); break; }
        // p0 (t x nb, column-major) = A64^T Y64, with A64 stored l x t and Y64 l x nb
        rc = gemm_tn_f64(p->device, st, sc.t, (int)nb, sc.l, (const double *)p->bat_a64, sc.l, y64, sc.l, p0, sc.t);
        if (rc != CSPD_OK) break;
        BatchArgs ba{};
        ba.b = nb;
        ba.p0 = p0;
        ba.g = (const float *)p->bat_g;
        ba.a64 = (const double *)p->bat_a64;
        ba.l = sc.l;
        ba.t = sc.t;
        ba.rank = a.fold == kDense ? a.m_dense : sc.l;
        ba.kvec = a.kvec ? a.kvec + b0 : nullptr;
        ba.kuni = a.kuni;
        ba.kcap = a.sup_count;
        ba.support = a.sup_out + b0 * a.sup_stride;
        ba.coef = (float *)a.coef_out + b0 * a.sup_stride;
        ba.k_used = a.kused_out + b0;
        ba.xhat = a.xhat ? (float *)a.xhat + b0 * (int64_t)a.n : nullptr;
        ba.dh = (const float *)p->d_high;
        ba.n = a.n;
        rc = kmax <= 16 ? by_n<16, false>(ba, sc.t, a.scale, st) : by_n<64, false>(ba, sc.t, a.scale, st);
        if (rc != CSPD_OK && !has_error()) rc = set_error(rc, "batch OMP kernel launch failed");
    }
    (void)hipFreeAsync(ws, st);
    return rc;
}

}  // namespace cspd
