// Plan-time kernels: effective dictionaries A_s = Phi U D_s (Section III-C,
// problems (P_low) and (P_high)), their squared column norms and, for small
// shared dictionaries, their Gram matrices.  Everything is formed in FP64 and
// rounded once to the plan's dtype.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "cspd_internal.h"

namespace cspd {
namespace {

// A64[t][i] = sum_j phi[i][j] * D[map[j]][t]   (t < T, i < M), FP64.
__global__ void k_eff_dense(const double *__restrict__ dict, int ns, int t_atoms,
                            const double *__restrict__ phi, int m, int n,
                            const int *__restrict__ map, double *__restrict__ a64)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t_atoms * m) return;
    int t = (int)(idx / m);
    int i = (int)(idx % m);
    const double *d = dict + (int64_t)t * ns;
    const double *row = phi + (int64_t)i * n;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc = fma(row[j], d[map[j]], acc);
    a64[idx] = acc;
}

// Folded candidates: A64[t][j] = D[j][t] (unweighted, the scale's own
// coordinates) and W64[t][j] = sqrt(w_j) D[j][t] with w_j the block size.
__global__ void k_fold_copy(const double *__restrict__ dict, int ns, int t_atoms,
                            const double *__restrict__ sqw, double *__restrict__ a64,
                            double *__restrict__ w64)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t_atoms * ns) return;
    int j = (int)(idx % ns);
    a64[idx] = dict[idx];
    if (w64) w64[idx] = sqw[j] * dict[idx];
}

template <typename T>
__global__ void k_cast_rows(const double *__restrict__ src, int t_atoms, int l, T *__restrict__ dst,
                            int lp)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t_atoms * lp) return;
    int t = (int)(idx / lp);
    int i = (int)(idx % lp);
    dst[idx] = i < l ? (T)src[(int64_t)t * l + i] : (T)0;
}

__global__ void k_cast_rows_lo(const double *__restrict__ src, int t_atoms, int l,
                               uint16_t *__restrict__ dst, int lp, int bf16)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t_atoms * lp) return;
    int t = (int)(idx / lp);
    int i = (int)(idx % lp);
    float f = i < l ? (float)src[(int64_t)t * l + i] : 0.0f;
    uint16_t h;
    if (bf16) {
        uint32_t u = __float_as_uint(f);
        u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
        h = (uint16_t)(u >> 16);
    } else {
        _Float16 v = (_Float16)f;
        h = *reinterpret_cast<uint16_t *>(&v);
    }
    dst[idx] = h;
}

// Two-term FP16 split of s v (s a power of two), for the matrix-core Gram:
// h = fp16(s v) (nearest), l = fp16(s v - h) (s v - h is exact in FP32).
// Row layout (lp 32-bit words per atom): per 8 coordinates, the four pairs of
// high parts, then the four pairs of low parts.
__global__ void k_split_rows(const float *__restrict__ v, int t_atoms, int lp, float s,
                             uint32_t *__restrict__ out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t_atoms * lp) return;
    const int t = (int)(idx / lp);
    const int w = (int)(idx % lp);
    const int k = w & 7;
    const int j = (w & ~7) + 2 * (k & 3);   // first coordinate of the pair
    const float *row = v + (int64_t)t * lp;
    uint32_t word = 0;
    for (int e = 0; e < 2; ++e) {
        const float x = row[j + e] * s;
        const _Float16 h = (_Float16)x;
        const _Float16 part = k < 4 ? h : (_Float16)(x - (float)h);
        const uint32_t bits = __builtin_bit_cast(uint16_t, part);
        word |= bits << (16 * e);
    }
    out[idx] = word;
}

template <typename T>
__global__ void k_norms(const double *__restrict__ w64, int t_atoms, int l, T *__restrict__ nu2)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t_atoms) return;
    const double *a = w64 + (int64_t)t * l;
    double s = 0.0;
    for (int i = 0; i < l; ++i) s = fma(a[i], a[i], s);
    nu2[t] = (T)s;
}

__global__ void k_inv_norms(const double *__restrict__ w64, int t_atoms, int l, float *__restrict__ inv)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t_atoms) return;
    const double *a = w64 + (int64_t)t * l;
    double s = 0.0;
    for (int i = 0; i < l; ++i) s = fma(a[i], a[i], s);
    inv[t] = s > 0.0 ? (float)(1.0 / sqrt(s)) : -1.0f;   // negative: never selectable
}

template <typename T>
__global__ void k_gram(const double *__restrict__ w64, int t_atoms, int l, T *__restrict__ g)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t_atoms * t_atoms) return;
    int a = (int)(idx / t_atoms);
    int b = (int)(idx % t_atoms);
    const double *x = w64 + (int64_t)a * l;
    const double *y = w64 + (int64_t)b * l;
    double s = 0.0;
    for (int i = 0; i < l; ++i) s = fma(x[i], y[i], s);
    g[idx] = (T)s;
}

// Largest |entry| of n values (one workgroup of 256; plan time only).
__global__ void k_absmax(const double *__restrict__ a, int64_t n, double *__restrict__ out)
{
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(a[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }


template <typename T>
cspd_status finish_scale(ScalePlan &sc, const double *a64, const double *w64, bool want_norms,
                         bool want_gram, int want_lo, int phases, hipStream_t st, int64_t &bytes)
{
    const int bs = 256;
    // one block of t rows per operator phase
    const int rows = sc.t * phases;
    size_t vbytes = sizeof(T) * (size_t)rows * sc.lp;
    CSPD_HIP_CHECK(hipMalloc(&sc.v, vbytes));
    bytes += vbytes;
    k_cast_rows<T><<<blocks_for((int64_t)rows * sc.lp, bs), bs, 0, st>>>(a64, rows, sc.l, (T *)sc.v, sc.lp);
    CSPD_HIP_CHECK(hipGetLastError());
    if (want_lo) {
        size_t lb = sizeof(uint16_t) * (size_t)sc.t * sc.lp;
        CSPD_HIP_CHECK(hipMalloc(&sc.v_lo, lb));
        bytes += lb;
        k_cast_rows_lo<<<blocks_for((int64_t)sc.t * sc.lp, bs), bs, 0, st>>>(
            a64, sc.t, sc.l, (uint16_t *)sc.v_lo, sc.lp, want_lo == CSPD_CORR_BF16_RESCORE);
        CSPD_HIP_CHECK(hipGetLastError());
    }
    if (want_norms) {
        // t entries per operator phase (w64 holds the phases' rows back to back)
        CSPD_HIP_CHECK(hipMalloc(&sc.nu2, sizeof(T) * (size_t)rows));
        bytes += sizeof(T) * (size_t)rows;
        k_norms<T><<<blocks_for(rows, bs), bs, 0, st>>>(w64, rows, sc.l, (T *)sc.nu2);
        CSPD_HIP_CHECK(hipGetLastError());
        CSPD_HIP_CHECK(hipMalloc(&sc.inv_nu, sizeof(float) * (size_t)rows));
        bytes += sizeof(float) * (size_t)rows;
        k_inv_norms<<<blocks_for(rows, bs), bs, 0, st>>>(w64, rows, sc.l, (float *)sc.inv_nu);
        CSPD_HIP_CHECK(hipGetLastError());
    }
    if (want_gram) {
        // one t x t table per operator phase (w64 holds the phases' rows back to back)
        size_t gb = sizeof(T) * (size_t)sc.t * sc.t * phases;
        CSPD_HIP_CHECK(hipMalloc(&sc.gram, gb));
        bytes += gb;
        for (int ph = 0; ph < phases; ++ph) {
            k_gram<T><<<blocks_for((int64_t)sc.t * sc.t, bs), bs, 0, st>>>(
                w64 + (size_t)ph * sc.t * sc.l, sc.t, sc.l, (T *)sc.gram + (size_t)ph * sc.t * sc.t);
            CSPD_HIP_CHECK(hipGetLastError());
        }
    }
    return CSPD_OK;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

cspd_status plan_effective(cspd_plan_s *p, const cspd_plan_desc *d, hipStream_t st)
{
    const int S = p->s, N = p->n, M = p->m;
    const int P = p->n_phases;
    // composed maps: finest coordinate -> scale-s coordinate
    std::vector<std::vector<int>> maps(S, std::vector<int>(N));
    for (int j = 0; j < N; ++j) maps[S - 1][j] = j;
    for (int s = S - 2; s >= 0; --s)
        for (int j = 0; j < N; ++j) maps[s][j] = d->up_map[s][maps[s + 1][j]];

    DevBuf phi_d;
    if (p->phi_kind == CSPD_PHI_DENSE) {
        CSPD_HIP_CHECK(hipMalloc(&phi_d.p, sizeof(double) * (size_t)P * M * N));
        CSPD_HIP_CHECK(hipMemcpyAsync(phi_d.p, d->phi, sizeof(double) * (size_t)P * M * N,
                                      hipMemcpyHostToDevice, st));
    }
    for (int s = 0; s < S; ++s) {
        cspd::ScalePlan &sc = p->sc[s];
        const int ns = d->dim[s], T = d->atoms[s];
        DevBuf dict_d, map_d, a64, w64, sqw_d;
        CSPD_HIP_CHECK(hipMalloc(&dict_d.p, sizeof(double) * (size_t)ns * T));
        CSPD_HIP_CHECK(hipMemcpyAsync(dict_d.p, d->dict[s], sizeof(double) * (size_t)ns * T,
                                      hipMemcpyHostToDevice, st));
        const bool dense = p->phi_kind == CSPD_PHI_DENSE;
        const bool mask = p->phi_kind == CSPD_PHI_MASK;
        const int l = dense ? M : ns;
        CSPD_HIP_CHECK(hipMalloc(&a64.p, sizeof(double) * (size_t)l * T * P));
        std::vector<int> off(ns + 1, 0), idx(N);
        std::vector<double> sqw(ns, 0.0);
        if (dense) {
            CSPD_HIP_CHECK(hipMalloc(&map_d.p, sizeof(int) * (size_t)N));
            CSPD_HIP_CHECK(hipMemcpyAsync(map_d.p, maps[s].data(), sizeof(int) * (size_t)N,
                                          hipMemcpyHostToDevice, st));
            for (int ph = 0; ph < P; ++ph) {
                k_eff_dense<<<blocks_for((int64_t)T * M, 256), 256, 0, st>>>(
                    (const double *)dict_d.p, ns, T, (const double *)phi_d.p + (size_t)ph * M * N, M, N,
                    (const int *)map_d.p, (double *)a64.p + (size_t)ph * T * M);
                CSPD_HIP_CHECK(hipGetLastError());
            }
        } else {
            // block table of U for this scale (fine samples of each coarse one)
            for (int j = 0; j < N; ++j) off[maps[s][j] + 1]++;
            for (int t = 0; t < ns; ++t) off[t + 1] += off[t];
            std::vector<int> fill(off.begin(), off.end() - 1);
            for (int j = 0; j < N; ++j) idx[fill[maps[s][j]]++] = j;
            for (int t = 0; t < ns; ++t) sqw[t] = std::sqrt((double)(off[t + 1] - off[t]));
            CSPD_HIP_CHECK(hipMalloc(&sqw_d.p, sizeof(double) * (size_t)ns));
            CSPD_HIP_CHECK(hipMemcpyAsync(sqw_d.p, sqw.data(), sizeof(double) * (size_t)ns,
                                          hipMemcpyHostToDevice, st));
            if (!mask) CSPD_HIP_CHECK(hipMalloc(&w64.p, sizeof(double) * (size_t)l * T));
            k_fold_copy<<<blocks_for((int64_t)T * ns, 256), 256, 0, st>>>(
                (const double *)dict_d.p, ns, T, (const double *)sqw_d.p, (double *)a64.p,
                (double *)w64.p);
            CSPD_HIP_CHECK(hipGetLastError());
            CSPD_HIP_CHECK(hipMalloc((void **)&sc.blk_off, sizeof(int) * (size_t)(ns + 1)));
            CSPD_HIP_CHECK(hipMalloc((void **)&sc.blk_idx, sizeof(int) * (size_t)N));
            CSPD_HIP_CHECK(hipMemcpyAsync(sc.blk_off, off.data(), sizeof(int) * (size_t)(ns + 1),
                                          hipMemcpyHostToDevice, st));
            CSPD_HIP_CHECK(hipMemcpyAsync(sc.blk_idx, idx.data(), sizeof(int) * (size_t)N,
                                          hipMemcpyHostToDevice, st));
            p->bytes += sizeof(int) * (size_t)(ns + 1 + N);
            bool ident = ns == N;
            for (int j = 0; ident && j < N; ++j) ident = idx[j] == j;
            sc.blk_ident = ident ? 1 : 0;
        }
        sc.n_s = ns;
        sc.t = T;
        sc.q = s == 0 ? 1 : T / d->atoms[s - 1];
        sc.l = l;
        sc.lp = 16;
        while (sc.lp < l) sc.lp *= 2;   // row stride = the kernels' register bucket
        sc.fold = dense ? kDense : kFold;
        // scale of the matrix-core Gram's FP16 split: the largest weighted
        // candidate entry (|v| times the square root of the largest block)
        // becomes at most 2^14, well inside FP16's range
        DevBuf amax_d;
        CSPD_HIP_CHECK(hipMalloc(&amax_d.p, sizeof(double)));
        k_absmax<<<1, 256, 0, st>>>((const double *)a64.p, (int64_t)l * T * P, (double *)amax_d.p);
        CSPD_HIP_CHECK(hipGetLastError());
        double vmax = 0.0;
        CSPD_HIP_CHECK(hipMemcpyAsync(&vmax, amax_d.p, sizeof(double), hipMemcpyDeviceToHost, st));
        CSPD_HIP_CHECK(hipStreamSynchronize(st));
        int cmax = 1;
        if (!dense)
            for (int t = 0; t < ns; ++t) cmax = std::max(cmax, off[t + 1] - off[t]);
        const double xmax = vmax * std::sqrt((double)cmax);
        int ex = 11;
        if (xmax > 0.0 && std::isfinite(xmax)) {
            ex = (int)std::floor(std::log2(16384.0 / xmax));
            ex = std::min(60, std::max(-60, ex));   // its square stays a normal float
        }
        sc.gsplit = std::ldexp(1.0f, ex);
        const double *wsrc = dense ? (const double *)a64.p : (const double *)w64.p;
        // Gram tables: one per operator; with several operators only at the
        // first scale (a full search there), within 64 MB
        const bool gram = !mask && T <= kMaxGramAtoms && sc.lp <= kMaxShortLen &&
                          ((P == 1 && (s == 0 || s == S - 1)) ||
                           (P > 1 && s == 0 && (int64_t)P * T * T * 4 <= ((int64_t)64 << 20)));
        // squared norms: one set per operator, with several operators only
        // beside the first scale's Gram tables (the batched correlations'
        // path); the 16-bit copy exists for a shared operator only
        const bool norms = !mask && (P == 1 || gram);
        // 16-bit copies for the reduced-precision proxy: full search at the
        // finest scale, and the first scale's batched contraction under a
        // shared dense operator
        const bool lo_scale = s == S - 1 || (s == 0 && dense && S >= 2);
        const int lo = (lo_scale && p->dtype == CSPD_F32 && P == 1) ? p->corr_mode : 0;
        cspd_status rc = p->dtype == CSPD_F64
            ? finish_scale<double>(sc, (const double *)a64.p, wsrc, norms, gram, 0, P, st, p->bytes)
            : finish_scale<float>(sc, (const double *)a64.p, wsrc, norms, gram, lo, P, st, p->bytes);
        if (rc != CSPD_OK) return rc;
        sc.phase_stride = (int64_t)T * sc.lp;
        // candidates whose per-patch weights are 0 or 1 (a shared dense
        // operator, or coarse samples that are single fine samples) are split
        // for the matrix-core Gram once here instead of in every patch
        if (p->dtype == CSPD_F32 && sc.lp >= 16 && sc.lp <= 128 && (dense || sc.blk_ident)) {
            const size_t sb = sizeof(uint32_t) * (size_t)sc.t * P * sc.lp;
            CSPD_HIP_CHECK(hipMalloc(&sc.v_split, sb));
            p->bytes += (int64_t)sb;
            k_split_rows<<<blocks_for((int64_t)sc.t * P * sc.lp, 256), 256, 0, st>>>(
                (const float *)sc.v, sc.t * P, sc.lp, sc.gsplit, (uint32_t *)sc.v_split);
            CSPD_HIP_CHECK(hipGetLastError());
        }
        if (s == S - 1 && p->dtype == CSPD_F32 && P == 1 && !mask && T <= kMaxBatchAtoms &&
            (p->k_max > kMaxK || T > 4096 || (T > kMaxLongCand && sc.lp > 128) || sc.lp > kMaxShortLen)) {
            // search in coefficient coordinates (full OMP over large
            // dictionaries or sparsities, and zero-tree OMP's finest scale on
            // long vectors): the effective atoms in FP64 and their Gram
            // matrix (FP64 GEMM, stored FP32)
            const size_t ab = sizeof(double) * (size_t)T * l;
            CSPD_HIP_CHECK(hipMalloc(&p->bat_a64, ab));
            p->bytes += (int64_t)ab;
            CSPD_HIP_CHECK(hipMemcpyAsync(p->bat_a64, a64.p, ab, hipMemcpyDeviceToDevice, st));
            DevBuf g64;
            CSPD_HIP_CHECK(hipMalloc(&g64.p, sizeof(double) * (size_t)T * T));
            const cspd_status grc = gemm_tn_f64(p->device, st, T, T, l, (const double *)a64.p, l,
                                                (const double *)a64.p, l, (double *)g64.p, T);
            if (grc != CSPD_OK) return grc;
            CSPD_HIP_CHECK(hipMalloc(&p->bat_g, sizeof(float) * (size_t)T * T));
            p->bytes += (int64_t)(sizeof(float) * (size_t)T * T);
            k_cast_rows<float><<<blocks_for((int64_t)T * T, 256), 256, 0, st>>>((const double *)g64.p, T, T,
                                                                                (float *)p->bat_g, T);
            CSPD_HIP_CHECK(hipGetLastError());
            CSPD_HIP_CHECK(hipStreamSynchronize(st));
        }
        if (s == S - 1) {
            // D_high in signal coordinates, atom-contiguous, for x-hat
            size_t eb = p->dtype == CSPD_F64 ? sizeof(double) : sizeof(float);
            CSPD_HIP_CHECK(hipMalloc(&p->d_high, eb * (size_t)T * N));
            p->bytes += eb * (size_t)T * N;
            if (p->dtype == CSPD_F64)
                k_cast_rows<double><<<blocks_for((int64_t)T * N, 256), 256, 0, st>>>(
                    (const double *)dict_d.p, T, N, (double *)p->d_high, N);
            else
                k_cast_rows<float><<<blocks_for((int64_t)T * N, 256), 256, 0, st>>>(
                    (const double *)dict_d.p, T, N, (float *)p->d_high, N);
            CSPD_HIP_CHECK(hipGetLastError());
        }
        // temporaries are freed at scope exit; make sure the kernels are done
        CSPD_HIP_CHECK(hipStreamSynchronize(st));
    }
    return CSPD_OK;
}

}  // namespace cspd
