// Per-patch OMP over long candidate vectors (more than 256 coordinates, up
// to 2048): the paper's 24x24 RGB image patches, 8x8x32 video patches and
// 4x4x8x8 light-field patches (Section IV), at any scale of the cross-scale
// model (Algorithm 2) or over every atom (Algorithm 1).
//
// One workgroup of 256 threads owns one patch and runs Algorithm 1 in the
// scale's coordinates, with the same operator folding as the short-vector
// kernels (identity and mask operators: candidates are D_s columns weighted
// per patch by the square root of the observed samples in each block; a
// shared dense operator: the plan's A_s = Phi U D_s):
//   proxy    every live candidate's |<a_i, r>| / ||a_i|| (FP32 dot products
//            over the coordinates, one wavefront per candidate at a time);
//   argmax   largest score, lowest atom index on exact ties;
//   merge    the new atom's Gram column against the support, its correlation
//            with y and its squared norm as FP64 sums of products of the
//            stored values, then the Cholesky row appended in FP64; an atom
//            whose pivot is at most 1e-10 of its squared norm is dependent
//            and ends the patch's selection;
//   project  L L^T alpha = A_Omega^T y by two FP64 triangular solves;
//   residue  r = y - A_Omega alpha, summed in FP64 and kept in FP32.
// The least squares are thus FP64 on the stored (rounded) vectors, as in the
// FP64 oracle; only the proxy is FP32.  Patches with at most 64 candidates
// (the finer scales of Algorithm 2) take the Gram mode further down, which
// reads each candidate once and iterates on the candidates' Gram matrix.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>

#include "cspd_internal.h"

namespace cspd {
namespace long_impl {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int KX = kMaxK;
constexpr int kCG = 8;   // candidates a wavefront scores at a time (their loads in flight together)

// LMAX coordinates and CMAX candidates at most: the launch picks the smallest
// instance that holds the scale, since LDS bounds the workgroups per CU
template <typename T, int LMAX, int CMAX>
struct Shared {
    alignas(16) T yhat[LMAX];   // measurement in the scale's coordinates
    alignas(16) T sqw[LMAX];    // per-coordinate weight (square root of observed samples)
    alignas(16) T rw[LMAX];     // weighted residual sqw * r
    int cand[CMAX];             // atom of each candidate slot; -1 once chosen or unusable
    T inv_nu[CMAX];             // reciprocal weighted norm of each candidate
    double L[KX * KX];       // Cholesky factor of the support's Gram matrix (row-major)
    double z[KX];
    double alpha[KX];
    int sup[KX];
    double red[kWaves][KX + 2];
    T wbest[kWaves];
    int wslot[kWaves];
    int count;
    int pick;                // candidate slot picked this iteration, -1 to stop
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v);

// Row-local DPP moves (quad xor 1 and 2, half-row mirror, row mirror) sum a
// value over each row of 16 lanes; permlane16 and permlane32 swaps then add
// the partner rows.  Every lane of the wavefront must be active (the callers
// loop over wavefront-uniform bounds); every lane ends with the sum.
template <int CTRL>
__device__ __forceinline__ int dpp_row(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ float sum_pairs(float v)
{
    auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
    v = __int_as_float(r16[0]) + __int_as_float(r16[1]);
    auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
    return __int_as_float(r32[0]) + __int_as_float(r32[1]);
}

template <>
__device__ __forceinline__ float wave_sum<float>(float v)
{
    v += __int_as_float(dpp_row<0xB1>(__float_as_int(v)));
    v += __int_as_float(dpp_row<0x4E>(__float_as_int(v)));
    v += __int_as_float(dpp_row<0x141>(__float_as_int(v)));
    v += __int_as_float(dpp_row<0x140>(__float_as_int(v)));
    return sum_pairs(v);
}

template <int CTRL>
__device__ __forceinline__ double dpp_row_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_row<CTRL>((int)b), hi = dpp_row<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ void swap_d(double v, bool wide, double &a, double &b)
{
    const long long bits = __double_as_longlong(v);
    int l0, l1, h0, h1;
    if (wide) {
        auto rl = __builtin_amdgcn_permlane32_swap((int)bits, (int)bits, false, false);
        auto rh = __builtin_amdgcn_permlane32_swap((int)(bits >> 32), (int)(bits >> 32), false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    } else {
        auto rl = __builtin_amdgcn_permlane16_swap((int)bits, (int)bits, false, false);
        auto rh = __builtin_amdgcn_permlane16_swap((int)(bits >> 32), (int)(bits >> 32), false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    }
    a = __longlong_as_double(((long long)h0 << 32) | (unsigned)l0);
    b = __longlong_as_double(((long long)h1 << 32) | (unsigned)l1);
}

template <>
__device__ __forceinline__ double wave_sum<double>(double v)
{
    v += dpp_row_d<0xB1>(v);
    v += dpp_row_d<0x4E>(v);
    v += dpp_row_d<0x141>(v);
    v += dpp_row_d<0x140>(v);
    double x, y;
    swap_d(v, false, x, y);
    v = x + y;
    swap_d(v, true, x, y);
    return x + y;
}

// Measurement of patch b in the scale's coordinates (yhat) and the weight of
// each coordinate (sqw: the square root of the observed fine samples folded
// into it; 1 or 0 without blocks); st_y and st_c (n entries each) stage the
// observed fine samples of block folds, or are null to read them in place.  *count (zeroed here) receives the
// coordinates of nonzero weight once the caller's next barrier has passed.
template <typename T>
__device__ void measure(const ScaleArgs &a, int64_t b, T *yhat, T *sqw, T *st_y, T *st_c, int *count)
{
    const int tid = threadIdx.x;
    const T *y = (const T *)a.y + b * (int64_t)a.y_stride;
    const int lp = a.lp, l = a.l;
    const bool fold = a.fold == kFold;
    const uint8_t *mrow = (fold && a.mask) ? a.mask + b * (int64_t)a.n : nullptr;
    if (tid == 0) *count = 0;
    if (!fold) {
        for (int t = tid; t < lp; t += kThreads) {
            yhat[t] = t < l ? y[t] : T(0);
            sqw[t] = t < l ? T(1) : T(0);
        }
    } else if (a.blk_ident) {
        for (int t = tid; t < lp; t += kThreads) {
            const bool obs = t < l && (mrow ? mrow[t] != 0 : true);
            yhat[t] = obs ? y[t] : T(0);
            sqw[t] = obs ? T(1) : T(0);
        }
    } else if (!st_y) {
        // blocks of several fine samples, read in place: each coordinate
        // folds its block (sum / sqrt(count), weight sqrt(count))
        for (int t = tid; t < lp; t += kThreads) {
            T cnt = 0, acc = 0;
            if (t < l) {
                for (int jj = a.blk_off[t]; jj < a.blk_off[t + 1]; ++jj) {
                    const int j = a.blk_idx[jj];
                    const bool obs = mrow ? mrow[j] != 0 : true;
                    cnt += obs ? T(1) : T(0);
                    acc += obs ? y[j] : T(0);
                }
            }
            const T sq = sqrt(cnt);
            yhat[t] = cnt > T(0) ? acc / sq : T(0);
            sqw[t] = sq;
        }
    } else {
        // blocks of several fine samples: stage the observed samples, then
        // each coordinate folds its block (sum / sqrt(count), weight sqrt(count))
        for (int j = tid; j < a.n; j += kThreads) {
            const bool obs = mrow ? mrow[j] != 0 : true;
            st_y[j] = obs ? y[j] : T(0);
            st_c[j] = obs ? T(1) : T(0);
        }
        __syncthreads();
        for (int t = tid; t < lp; t += kThreads) {
            T cnt = 0, acc = 0;
            if (t < l) {
                for (int jj = a.blk_off[t]; jj < a.blk_off[t + 1]; ++jj) {
                    const int j = a.blk_idx[jj];
                    cnt += st_c[j];
                    acc += st_y[j];
                }
            }
            const T sq = sqrt(cnt);
            yhat[t] = cnt > T(0) ? acc / sq : T(0);
            sqw[t] = sq;
        }
    }
    __syncthreads();
    int c = 0;
    for (int t = tid; t < lp; t += kThreads) c += sqw[t] > T(0);
    atomicAdd(count, c);
}

// Candidate atoms of patch b: every atom at the first scale, else the
// children of the previous scale's support (Algorithm 2), at most cap of
// them (the launch sizes cap to the largest count).  Returns how many.
__device__ int candidates(const ScaleArgs &a, int64_t b, int *cand, int cap)
{
    const int tid = threadIdx.x;
    int nc = a.first ? a.t : a.prev_kused[b] * a.q;
    nc = nc < cap ? nc : cap;
    if (a.first) {
        for (int i = tid; i < nc; i += kThreads) cand[i] = i;
        return nc;
    }
    for (int i = tid; i < nc; i += kThreads) {
        const int pj = i / a.q;
        const int parent = a.prev_sup[b * (int64_t)a.prev_stride + pj];
        cand[i] = parent * a.q + (i - pj * a.q);
    }
    return nc;
}

template <typename T, int LMAX, int CMAX, int CG>
__global__ __launch_bounds__(kThreads) void k_omp_long(ScaleArgs a)
{
    static_assert(sizeof(T) == 4, "the candidate loops read FP32 rows as float4");
    __shared__ Shared<T, LMAX, CMAX> sh;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int64_t b = blockIdx.x;
    if (b >= a.b) return;
    // operator of the patch (plans with several); out of range: unsolved
    int ph = a.phase ? a.phase[b] : 0;
    const bool phok = ph >= 0 && ph < a.n_phases;
    ph = phok ? ph : 0;
    const T *v = (const T *)a.v + (int64_t)ph * a.phase_stride;
    const int lp = a.lp, l = a.l;
    const bool fold = a.fold == kFold;

    measure(a, b, sh.yhat, sh.sqw, (T *)nullptr, (T *)nullptr, &sh.count);
    const int nc = candidates(a, b, sh.cand, CMAX);
    for (int t = tid; t < lp; t += kThreads) sh.rw[t] = sh.sqw[t] * sh.yhat[t];
    __syncthreads();
    const int rank_bound = fold ? sh.count : a.m_dense;
    const int kreq = a.kvec ? a.kvec[b] : a.kuni;
    int K = kreq < nc ? kreq : nc;
    K = phok ? K : 0;
    K = K < a.sup_count ? K : a.sup_count;
    K = K < KX ? K : KX;
    K = K > 0 ? K : 0;

    // ---- weighted norms of the candidates (CG per wavefront at a time) ----
    const int l4 = (l + 3) >> 2;   // 16-byte groups that hold the used coordinates (rows are padded with zeros)
    const float4 *sqw4 = reinterpret_cast<const float4 *>(sh.sqw);
    const float4 *rw4 = reinterpret_cast<const float4 *>(sh.rw);
    for (int i0 = wv * CG; i0 < nc; i0 += kWaves * CG) {
        const float4 *vp[CG];
#pragma unroll
        for (int c = 0; c < CG; ++c)
            vp[c] = reinterpret_cast<const float4 *>(v + (int64_t)(i0 + c < nc ? sh.cand[i0 + c] : 0) * lp);
        float acc[CG] = {};
        for (int t4 = lane; t4 < l4; t4 += 64) {
            const float4 w = sqw4[t4];
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                const float4 x = vp[c][t4];
                const float a0 = x.x * w.x, a1 = x.y * w.y, a2 = x.z * w.z, a3 = x.w * w.w;
                acc[c] += a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
            }
        }
#pragma unroll
        for (int c = 0; c < CG; ++c) {
            const float s = wave_sum(acc[c]);
            if (lane == 0 && i0 + c < nc) sh.inv_nu[i0 + c] = s > 0.f ? 1.f / sqrtf(s) : -1.f;
        }
    }
    __syncthreads();
    for (int i = tid; i < nc; i += kThreads)
        if (!(sh.inv_nu[i] > T(0))) sh.cand[i] = -1;   // a zero effective column is never picked
    __syncthreads();

    // ---- iterations (Algorithm 1) ------------------------------------------
    int n = 0;
    for (int it = 0; it < K; ++it) {
        // proxy and argmax: each wavefront keeps its best (score, slot)
        T best = T(-1);
        int bslot = -1;
        for (int i0 = wv * CG; i0 < nc; i0 += kWaves * CG) {
            int at[CG];
            const float4 *vp[CG];
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                at[c] = i0 + c < nc ? sh.cand[i0 + c] : -1;
                vp[c] = reinterpret_cast<const float4 *>(v + (int64_t)(at[c] >= 0 ? at[c] : 0) * lp);
            }
            bool any = false;
#pragma unroll
            for (int c = 0; c < CG; ++c) any = any || at[c] >= 0;
            if (!any) continue;   // wavefront-uniform
            float acc[CG] = {};
            for (int t4 = lane; t4 < l4; t4 += 64) {
                const float4 r = rw4[t4];
#pragma unroll
                for (int c = 0; c < CG; ++c) {
                    const float4 x = vp[c][t4];
                    acc[c] += x.x * r.x + x.y * r.y + x.z * r.z + x.w * r.w;
                }
            }
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                const float sc = fabsf(wave_sum(acc[c])) * (at[c] >= 0 ? sh.inv_nu[i0 + c] : 0.f);
                const bool up = at[c] >= 0 && (bslot < 0 || sc > best || (sc == best && at[c] < sh.cand[bslot]));
                best = up ? sc : best;
                bslot = up ? i0 + c : bslot;
            }
        }
        if (lane == 0) {
            sh.wbest[wv] = best;
            sh.wslot[wv] = bslot;
        }
        __syncthreads();
        if (tid == 0) {
            int ps = -1;
            T pb = T(-1);
            for (int w = 0; w < kWaves; ++w) {
                const int s = sh.wslot[w];
                if (s < 0) continue;
                const T sc = sh.wbest[w];
                if (ps < 0 || sc > pb || (sc == pb && sh.cand[s] < sh.cand[ps])) {
                    pb = sc;
                    ps = s;
                }
            }
            sh.pick = n < rank_bound ? ps : -1;   // candidates exhausted, or the support spans the space
        }
        __syncthreads();
        const int ps = sh.pick;
        if (ps < 0) break;
        const int k = sh.cand[ps];
        // Gram column against the support, correlation with y, squared norm:
        // FP64 sums of the stored values' products
        double part[KX + 2];
#pragma unroll
        for (int j = 0; j < KX + 2; ++j) part[j] = 0.0;
        const T *vk = v + (int64_t)k * lp;
        for (int t = tid; t < l; t += kThreads) {
            const double w = (double)sh.sqw[t];
            const double xk = (double)vk[t] * w;
#pragma unroll
            for (int j = 0; j < KX; ++j)
                if (j < n) part[j] += xk * ((double)v[(int64_t)sh.sup[j] * lp + t] * w);
            part[KX] += xk * (double)sh.yhat[t];
            part[KX + 1] += xk * xk;
        }
#pragma unroll
        for (int j = 0; j < KX + 2; ++j) {
            if (j < n || j >= KX) {
                const double s = wave_sum(part[j]);
                if (lane == 0) sh.red[wv][j] = s;
            }
        }
        __syncthreads();
        if (tid == 0) {
            double g[KX];
            for (int j = 0; j < n; ++j) g[j] = sh.red[0][j] + sh.red[1][j] + sh.red[2][j] + sh.red[3][j];
            const double hk = sh.red[0][KX] + sh.red[1][KX] + sh.red[2][KX] + sh.red[3][KX];
            const double ek = sh.red[0][KX + 1] + sh.red[1][KX + 1] + sh.red[2][KX + 1] + sh.red[3][KX + 1];
            // w = L^{-1} g; pivot ek - ||w||^2
            double d = ek;
            for (int i = 0; i < n; ++i) {
                double s = g[i];
                for (int j = 0; j < i; ++j) s -= sh.L[i * KX + j] * sh.L[n * KX + j];
                const double wi = s / sh.L[i * KX + i];
                sh.L[n * KX + i] = wi;
                d -= wi * wi;
            }
            if (!(d > 1e-10 * ek)) {
                sh.pick = -1;                 // dependent on the support
            } else {
                const double lnn = sqrt(d);
                sh.L[n * KX + n] = lnn;
                double s = hk;
                for (int j = 0; j < n; ++j) s -= sh.L[n * KX + j] * sh.z[j];
                sh.z[n] = s / lnn;
                // L^T alpha = z
                for (int i = n; i >= 0; --i) {
                    double u = sh.z[i];
                    for (int j = i + 1; j <= n; ++j) u -= sh.L[j * KX + i] * sh.alpha[j];
                    sh.alpha[i] = u / sh.L[i * KX + i];
                }
                sh.sup[n] = k;
                sh.cand[ps] = -1;
            }
        }
        __syncthreads();
        if (sh.pick < 0) break;
        ++n;
        // residue (weighted): sqw * (y - A_Omega alpha), summed in FP64
        for (int t = tid; t < lp; t += kThreads) {
            const double w = (double)sh.sqw[t];
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += sh.alpha[j] * (double)v[(int64_t)sh.sup[j] * lp + t];
            sh.rw[t] = (T)(w * ((double)sh.yhat[t] - w * s));
        }
        __syncthreads();
    }

    // ---- outputs -----------------------------------------------------------
    if (tid == 0) a.kused_out[b] = n;
    int *sup_out = a.sup_out + b * (int64_t)a.sup_stride;
    for (int i = tid; i < a.sup_count; i += kThreads) sup_out[i] = i < n ? sh.sup[i] : -1;
    if (!a.last) return;
    T *coef = (T *)a.coef_out + b * (int64_t)a.sup_stride;
    for (int i = tid; i < a.sup_count; i += kThreads) coef[i] = i < n ? (T)sh.alpha[i] : T(0);
    if (a.xhat) {
        const T *dh = (const T *)a.d_high;
        T *xh = (T *)a.xhat + b * (int64_t)a.n;
        for (int j = tid; j < a.n; j += kThreads) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += sh.alpha[i] * (double)dh[(int64_t)sh.sup[i] * a.n + j];
            xh[j] = (T)s;
        }
    }
}

// ---------------------------------------------------------------------------
// Gram mode: at most kGramCand candidates.  The patch's weighted candidate
// Gram matrix G = A^T W A (W: the squared coordinate weights) and the
// correlations h = A^T sqrt(W) yhat (yhat is the folded measurement, which
// carries the other factor) are formed once, as FP64 sums over the
// coordinates of nonzero weight only, from the candidates' stored values;
// Algorithm 1's steps then run on G and h alone (a precomputed Gram matrix,
// the usual way to speed up OMP when candidates are reused; not a step the
// paper prescribes): the proxy is c = h - G[:, Omega] alpha, the Cholesky row
// of a new atom reads its entries of G, and no candidate vector is read
// again.  Each
// candidate row leaves HBM once instead of once per iteration, and a mask
// leaves its unobserved coordinates out of the arithmetic.
//
// Formation: the observed coordinates are listed in ascending order; chunks
// of kCh of them are staged in LDS as FP64 weighted values (exact products
// of the FP32 candidate value and weight), the loads of the next kBuf
// chunks in flight while the current one is multiplied (the loop waits on
// gathers from beyond L2, not on arithmetic).  G is symmetric: its ten upper 16x16
// tiles are FP64 matrix-core products (16x16x4: one LDS double per lane per
// tile and step, where 4x4 register blocks on the vector units read eight
// per sixteen FMAs and waited on LDS), three tiles for each of three
// wavefronts and one for the fourth, which also forms h.  The roles rotate
// with the workgroup index.  Only the upper triangle is kept (packed rows).
constexpr int kGramCand = 64;
constexpr int kGramTri = kGramCand * (kGramCand + 1) / 2;
constexpr int kCh = 16;
constexpr int kBuf = 3;               // chunks whose loads are in flight
constexpr int kXld = kGramCand + 2;   // keeps rows 16-byte aligned and spreads the staging stores over banks
typedef double d4 __attribute__((ext_vector_type(4)));

// LDS by phase: the measurement and weights live until the list of
// observed coordinates is built, then their space holds the staged chunks;
// the list (16-bit coordinates, weights, measurement) lives through the
// formation, then its space holds the packed Gram matrix.
template <typename T>
struct GramShared {
    union {
        struct {
            T yhat[kMaxLongLen];
            T sqw[kMaxLongLen];
        } m;                            // measurement in the scale's coordinates and weights
        double X[kCh][kXld];            // staged chunk: weighted candidate values [coordinate][slot]
    } a;
    union {
        struct {
            unsigned short idx[kMaxLongLen];   // coordinates of nonzero weight, ascending
            T wc[kMaxLongLen];                 // their weights
            T yc[kMaxLongLen];                 // their measurement values
        } c;
        double G[kGramTri];             // packed upper triangle of the weighted Gram matrix
    } b;
    double yw[kCh];                     // yhat at the chunk's coordinates (already folded: one weight factor)
    double h[kGramCand];                // weighted correlations with the measurement
    int cand[kGramCand];
    double L[KX * KX];
    double z[KX];
    double alpha[KX];
    int sup[KX];
    int wcnt[kWaves];
    int count;
    int nsel;
};

__device__ __forceinline__ int tri(int i, int j)
{
    const int r = i < j ? i : j, c = i < j ? j : i;
    return r * kGramCand - ((r * (r - 1)) >> 1) + (c - r);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_omp_long_gram(ScaleArgs a)
{
    __shared__ GramShared<T> sh;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int64_t b = blockIdx.x;
    if (b >= a.b) return;
    int ph = a.phase ? a.phase[b] : 0;
    const bool phok = ph >= 0 && ph < a.n_phases;
    ph = phok ? ph : 0;
    const T *v = (const T *)a.v + (int64_t)ph * a.phase_stride;
    const int lp = a.lp;
    const bool fold = a.fold == kFold;
    // the wavefronts' roles in the formation rotate with the workgroup, so
    // that the workgroups sharing a CU do not load the same SIMDs
    const int role = (wv + (int)(b & 3)) & 3;

    measure(a, b, sh.a.m.yhat, sh.a.m.sqw, (T *)nullptr, (T *)nullptr, &sh.count);
    const int nc = candidates(a, b, sh.cand, kGramCand);

    // ---- observed coordinates, ascending (each wavefront a contiguous range)
    const int seg = ((lp + kThreads - 1) / kThreads) * 64;
    const int lo = wv * seg;
    {
        int c = 0;
        for (int t0 = lo; t0 < lo + seg; t0 += 64) {
            const int t = t0 + lane;
            c += __popcll(__ballot(t < lp && sh.a.m.sqw[t] > T(0)));
        }
        if (lane == 0) sh.wcnt[wv] = c;
    }
    __syncthreads();
    const int rank_bound = fold ? sh.count : a.m_dense;
    const int kreq = a.kvec ? a.kvec[b] : a.kuni;
    int K = kreq < nc ? kreq : nc;
    K = phok ? K : 0;
    K = K < a.sup_count ? K : a.sup_count;
    K = K < KX ? K : KX;
    K = K > 0 ? K : 0;
    int M = 0, base = 0;
    for (int w = 0; w < kWaves; ++w) {
        base += w < wv ? sh.wcnt[w] : 0;
        M += sh.wcnt[w];
    }
    for (int t0 = lo; t0 < lo + seg; t0 += 64) {
        const int t = t0 + lane;
        const bool o = t < lp && sh.a.m.sqw[t] > T(0);
        const unsigned long long m = __ballot(o);
        if (o) {
            const int p = base + __popcll(m & ((1ull << lane) - 1ull));
            sh.b.c.idx[p] = (unsigned short)t;
            sh.b.c.wc[p] = sh.a.m.sqw[t];
            sh.b.c.yc[p] = sh.a.m.yhat[t];
        }
        base += __popcll(m);
    }
    __syncthreads();

    if (K > 0) {
        // ---- G and h over the observed coordinates ---------------------------
        // staging: element e = tid + 256 r is slot e / kCh, chunk coordinate e % kCh
        constexpr int kPer = kGramCand * kCh / kThreads;
        const int spp = tid % kCh;
        const T *rowp[kPer];
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int i = (tid + r * kThreads) / kCh;
            rowp[r] = i < nc ? v + (int64_t)sh.cand[i] * lp : nullptr;
        }
        auto fetch_to = [&](T (&buf)[kPer], int &ptv, int p0) {
            const int p = p0 + spp;
            ptv = p < M ? p : -1;   // position in the list of observed coordinates
            const int t = ptv >= 0 ? (int)sh.b.c.idx[ptv] : 0;
#pragma unroll
            for (int r = 0; r < kPer; ++r) buf[r] = (ptv >= 0 && rowp[r]) ? rowp[r][t] : T(0);
        };
        // tiles of this wavefront's role: G's ten upper 16x16 tiles, three
        // each for roles 0-2, one for role 3 (which also forms h).  Tile t
        // is (ti, tj) = (kTile[role][t] >> 2, kTile[role][t] & 3).
        constexpr int kTile[4][3] = {{0, 1, 2}, {3, 5, 6}, {7, 10, 11}, {15, 15, 15}};
        const int ntile = role < 3 ? 3 : 1;
        int ti[3], tj[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int code = role == 0 ? kTile[0][t] : role == 1 ? kTile[1][t] : role == 2 ? kTile[2][t] : kTile[3][t];
            ti[t] = code >> 2;
            tj[t] = code & 3;
        }
        const int fi = lane & 15, fk = lane >> 4;   // operand lane: row (or column) fi of the tile, coordinate fk
        d4 acc[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
        double hacc = 0.0;

        // kBuf chunks in flight: each chunk's buffer is refilled with the chunk
        // kBuf ahead as soon as it has been staged
        auto run_chunk = [&](T (&buf)[kPer], int &ptv, int p0) {
            __syncthreads();   // the previous chunk has been consumed
            {
                const double w = ptv >= 0 ? (double)sh.b.c.wc[ptv] : 0.0;
#pragma unroll
                for (int r = 0; r < kPer; ++r) sh.a.X[spp][(tid + r * kThreads) / kCh] = (double)buf[r] * w;
                if (tid < kCh) sh.yw[tid] = ptv >= 0 ? (double)sh.b.c.yc[ptv] : 0.0;
            }
            __syncthreads();
            if (p0 + kBuf * kCh < M) fetch_to(buf, ptv, p0 + kBuf * kCh);
            // G tile (ti, tj) += X[k, 16 ti + 0..15]^T X[k, 16 tj + 0..15] over
            // the chunk's coordinates, four per matrix-core step
#pragma unroll
            for (int ks = 0; ks < kCh / 4; ++ks) {
                const double *xr = sh.a.X[4 * ks + fk];
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    if (t < ntile)   // wavefront-uniform
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[16 * ti[t] + fi], xr[16 * tj[t] + fi], acc[t],
                                                                      0, 0, 0);
                }
            }
            if (role == 3) {
#pragma unroll
                for (int pp = 0; pp < kCh; ++pp) hacc = fma(sh.a.X[pp][lane], sh.yw[pp], hacc);
            }
        };
        T buf[kBuf][kPer];
        int ptb[kBuf];
#pragma unroll
        for (int q = 0; q < kBuf; ++q) {
            ptb[q] = -1;
            if (q * kCh < M) fetch_to(buf[q], ptb[q], q * kCh);
        }
        for (int p0 = 0; p0 < M; p0 += kBuf * kCh) {
#pragma unroll
            for (int q = 0; q < kBuf; ++q)
                if (p0 + q * kCh < M) run_chunk(buf[q], ptb[q], p0 + q * kCh);
        }
        __syncthreads();   // the staging area and the measurement staging are free
        // result layout of the 16x16 FP64 tile (unlike the FP32 16x16 ones):
        // register r of lane l holds row 4 r + l / 16 of column l % 16
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (t < ntile) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = 16 * ti[t] + 4 * r + fk, gj = 16 * tj[t] + fi;
                    if (gi <= gj) sh.b.G[tri(gi, gj)] = acc[t][r];
                }
            }
        }
        if (role == 3) sh.h[lane] = hacc;
        __syncthreads();

        // ---- iterations in candidate coordinates (the role-3 wavefront) ------
        // Lane i keeps, for candidate slot i, u_i = L^-1 G[Omega, i] (the new
        // rows of the Cholesky factor it would add), its correlation with the
        // residual c_i = h_i - u_i^T z and its squared pivot e_i = G_ii -
        // ||u_i||^2, all FP64 in registers (the loop is unrolled, so the row
        // index is a constant).  A pick appends the chosen lane's
        // [u_k^T, sqrt(e_k)] to L; every lane then takes one more entry of u_i
        // (one dot product with u_k and a division) and updates c_i, e_i.
        // The coefficients are solved once, after the last pick.
        if (role == 3) {
            const int ci = lane < nc ? sh.cand[lane] : -1;
            const double gii = ci >= 0 ? sh.b.G[tri(lane, lane)] : 0.0;
            bool live = ci >= 0 && gii > 0.0;
            const double rn = live ? 1.0 / sqrt(gii) : 0.0;
            double c = sh.h[lane], e = gii;
            double u[KX];
#pragma unroll
            for (int j = 0; j < KX; ++j) u[j] = 0.0;
            int n = 0;
            // no early exit from the unrolled loop: a stop turns the rest off
#pragma unroll
            for (int it = 0; it < KX; ++it) {
                if (n < it || it >= K) continue;
                double sc = live ? fabs(c) * rn : -1.0;
                int at = live ? ci : INT_MAX;
                int ps = live ? lane : -1;
                // largest score, lowest atom index on exact ties
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const double os = __shfl_xor(sc, off);
                    const int oa = __shfl_xor(at, off);
                    const int op = __shfl_xor(ps, off);
                    const bool up = os > sc || (os == sc && oa < at);
                    sc = up ? os : sc;
                    at = up ? oa : at;
                    ps = up ? op : ps;
                }
                if (ps < 0 || it >= rank_bound) continue;   // candidates exhausted, or the support spans the space
                const double ek = __shfl(e, ps), gkk = __shfl(gii, ps);
                if (!(ek > 1e-10 * gkk)) continue;          // dependent on the support
                const double lnn = sqrt(ek);
                const double zn = __shfl(c, ps) / lnn;
                double uk[KX];
#pragma unroll
                for (int j = 0; j < it; ++j) uk[j] = __shfl(u[j], ps);
                double dot = 0.0;
#pragma unroll
                for (int j = 0; j < it; ++j) dot = fma(uk[j], u[j], dot);
                const double un = (live ? sh.b.G[tri(lane, ps)] - dot : 0.0) / lnn;
                u[it] = un;
                c = fma(-un, zn, c);
                e = fma(-un, un, e);
                if (lane == 0) {
#pragma unroll
                    for (int j = 0; j < it; ++j) sh.L[it * KX + j] = uk[j];
                    sh.L[it * KX + it] = lnn;
                    sh.z[it] = zn;
                    sh.sup[it] = at;
                }
                live = live && lane != ps;
                n = it + 1;
            }
            if (lane == 0) {
                // L^T alpha = z (lane 0 reads back only its own writes)
                for (int i = n - 1; i >= 0; --i) {
                    double v2 = sh.z[i];
                    for (int j = i + 1; j < n; ++j) v2 -= sh.L[j * KX + i] * sh.alpha[j];
                    sh.alpha[i] = v2 / sh.L[i * KX + i];
                }
                sh.nsel = n;
            }
        }
    } else if (tid == 0) {
        sh.nsel = 0;
    }
    __syncthreads();

    // ---- outputs -----------------------------------------------------------
    const int n = sh.nsel;
    if (tid == 0) a.kused_out[b] = n;
    int *sup_out = a.sup_out + b * (int64_t)a.sup_stride;
    for (int i = tid; i < a.sup_count; i += kThreads) sup_out[i] = i < n ? sh.sup[i] : -1;
    if (!a.last) return;
    T *coef = (T *)a.coef_out + b * (int64_t)a.sup_stride;
    for (int i = tid; i < a.sup_count; i += kThreads) coef[i] = i < n ? (T)sh.alpha[i] : T(0);
    if (a.xhat) {
        const T *dh = (const T *)a.d_high;
        T *xh = (T *)a.xhat + b * (int64_t)a.n;
        for (int j = tid; j < a.n; j += kThreads) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += sh.alpha[i] * (double)dh[(int64_t)sh.sup[i] * a.n + j];
            xh[j] = (T)s;
        }
    }
}

}  // namespace long_impl

bool long_fits(const ScaleArgs &a, int max_cand)
{
    return a.lp > 0 && a.lp <= kMaxLongLen && a.l <= kMaxLongLen && a.n <= kMaxLongLen && max_cand <= kMaxLongCand;
}

cspd_status launch_long(int dtype, const ScaleArgs &a, int max_cand, hipStream_t st)
{
    using namespace long_impl;
    if (a.b <= 0) return CSPD_OK;
    if (!long_fits(a, max_cand)) return CSPD_E_UNSUPPORTED;
    if (dtype != CSPD_F32) return CSPD_E_UNSUPPORTED;
    const bool gram = max_cand <= kGramCand;
    char label[96];
    if (a.first && a.last)
        snprintf(label, sizeof(label), "omp_long<f32,%slp%d>:full", gram ? "gram," : "", a.lp);
    else
        snprintf(label, sizeof(label), "omp_long<f32,%slp%d>:s%d", gram ? "gram," : "", a.lp, a.scale);
    const dim3 grid((unsigned)a.b), block(kThreads);
    if (gram)
        launch_timed(label, k_omp_long_gram<float>, grid, block, 0, st, a);
    else if (a.lp <= 512 && max_cand <= 256)
        launch_timed(label, k_omp_long<float, 512, 256, 4>, grid, block, 0, st, a);
    else
        launch_timed(label, k_omp_long<float, kMaxLongLen, kMaxLongCand, kCG>, grid, block, 0, st, a);
    CSPD_HIP_CHECK(hipGetLastError());
    return CSPD_OK;
}

}  // namespace cspd
