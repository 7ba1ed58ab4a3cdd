// Per-patch OMP over one scale of the cross-scale model.
//
// One wavefront owns one patch.  Lanes own candidate atoms (slot s of lane l
// is candidate s*64 + l); at scale 0 every atom of D_0 is a candidate
// (problem (P_low) of Section III-C), at finer scales the candidates are the
// child blocks f(Omega) of the previous scale's support (Section III-B,
// problem (P_high), Algorithm 2), in ascending atom order.
//
// The iteration is Algorithm 1 -- proxy, support merge, projection, residue
// -- carried in candidate coordinates with an incremental Cholesky factor:
//   u_i   = L^{-1} A_Omega^T a_i   (row n of L is appended when atom k joins:
//                                   [u_k^T, sqrt(e_k)])
//   c_i   = <a_i, r>   = h_i - u_i^T z,   z = L^{-1} A_Omega^T y
//   e_i   = ||(I - P_Omega) a_i||^2 = ||a_i||^2 - ||u_i||^2
// so each step costs one Gram column <a_i, a_k> per candidate plus rank-1
// updates of c, e and u; the residue r = y - A_Omega alpha is never formed,
// only its correlations with the candidates.  The least-squares coefficients
// alpha solve L^T alpha = z once the loop ends.
//
// Candidate vectors live in VGPRs (vec mode) or, when a shared operator makes
// the Gram matrix of a small dictionary patch-independent, the Gram column is
// read from the plan (gram mode).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>

#include "cspd_internal.h"

namespace cspd {
namespace {

constexpr int W = kWavesPerBlock;
constexpr int KM = kMaxK;
constexpr int LP_GRAM = 256;   // LDS row length for gram-mode kernels

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <typename T> __device__ __forceinline__ T dep_tol();
template <> __device__ __forceinline__ double dep_tol<double>() { return 1e-10; }
template <> __device__ __forceinline__ float dep_tol<float>() { return 1e-5f; }

template <typename T>
__device__ __forceinline__ void wave_argmax(T &best, int &idx)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T ob = __shfl_xor(best, off);
        int oi = __shfl_xor(idx, off);
        if (ob > best || (ob == best && oi < idx)) { best = ob; idx = oi; }
    }
}

template <typename T, int LPA>
struct WaveLds {
    T yhat[LPA];
    T sqw[LPA];
    T vk[LPA];
    T uk[KM];
    T sc[4];
    T z[KM];
    T alpha[KM];
    T lmat[KM][KM + 1];
    int sup[KM];
    int par[KM];
};

// FP64 Gram matrix and right-hand side of the atoms ids[0..n-1], accumulated
// in FP64 from the stored vectors (lanes split the n(n+1)/2 + n dot
// products), then, on lane 0, an FP64 Cholesky factorisation in place and,
// when `solve`, the forward and back substitutions (solution left in h64).
// diag_before[j] keeps G_jj before factoring.  Used by FP32 plans for the
// pivot and the back-substitution of ill-conditioned supports.
template <typename T, int LPA>
__device__ void gram64_chol(WaveLds<T, LPA> &w, const ScaleArgs &a, const int *ids, int n, int lane,
                            double *g64, double *h64, double *diag_before, bool solve)
{
    const T *v = (const T *)a.v;
    const int np = n * (n + 1) / 2;
    for (int pidx = lane; pidx < np + n; pidx += 64) {
        double s = 0.0;
        if (pidx < np) {
            int i = 0, rem = pidx;
            while (rem > i) { rem -= i + 1; ++i; }
            const int j = rem;  // j <= i
            const T *vi = v + (int64_t)ids[i] * a.lp;
            const T *vj = v + (int64_t)ids[j] * a.lp;
            for (int t = 0; t < a.l; ++t) {
                const double wt = (double)w.sqw[t];
                s += ((double)vi[t] * wt) * ((double)vj[t] * wt);
            }
            g64[i * KM + j] = s;
            g64[j * KM + i] = s;
        } else {
            const int i = pidx - np;
            const T *vi = v + (int64_t)ids[i] * a.lp;
            for (int t = 0; t < a.l; ++t) s += (double)vi[t] * (double)w.sqw[t] * (double)w.yhat[t];
            h64[i] = s;
        }
    }
    wave_sync();
    if (lane == 0) {
        for (int j = 0; j < n; ++j) diag_before[j] = g64[j * KM + j];
        for (int j = 0; j < n; ++j) {
            double d = g64[j * KM + j];
            for (int k = 0; k < j; ++k) d -= g64[j * KM + k] * g64[j * KM + k];
            g64[j * KM + j] = d;                      // pivot (squared diagonal) kept for the caller
            const double r = d > 0.0 ? sqrt(d) : 0.0;
            for (int i = j + 1; i < n; ++i) {
                double t = g64[i * KM + j];
                for (int k = 0; k < j; ++k) t -= g64[i * KM + k] * g64[j * KM + k];
                g64[i * KM + j] = r > 0.0 ? t / r : 0.0;
            }
            g64[j * KM + j] = r;
            diag_before[KM + j] = d;
        }
        if (solve) {
            for (int i = 0; i < n; ++i) {
                double t = h64[i];
                for (int k = 0; k < i; ++k) t -= g64[i * KM + k] * h64[k];
                h64[i] = g64[i * KM + i] > 0.0 ? t / g64[i * KM + i] : 0.0;
            }
            for (int i = n - 1; i >= 0; --i) {
                double t = h64[i];
                for (int k = i + 1; k < n; ++k) t -= g64[k * KM + i] * h64[k];
                h64[i] = g64[i * KM + i] > 0.0 ? t / g64[i * KM + i] : 0.0;
            }
        }
    }
    wave_sync();
}

// Condition estimate of G = L L^T from its factor: tr(G) tr(G^{-1}) / n, which
// lies between kappa(G) / n and n kappa(G).  tr(G^{-1}) = ||L^{-1}||_F^2; lane
// j forms column j of L^{-1} by forward substitution (static indexing, so the
// column stays in registers).
template <typename T, int LPA>
__device__ double cond_estimate(const WaveLds<T, LPA> &w, int n, int lane)
{
    double col2 = 0.0, tr = 0.0;
    double x[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) {
        x[i] = 0.0;
        if (i < n) {
            double t = (i == lane) ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < i; ++m) t -= (double)w.lmat[i][m] * x[m];
            x[i] = t / (double)w.lmat[i][i];
            if (lane < n) col2 += x[i] * x[i];
            double rr = 0.0;
#pragma unroll
            for (int m = 0; m <= i; ++m) rr += (double)w.lmat[i][m] * (double)w.lmat[i][m];
            tr += rr;                                  // sum of G_ii = ||row i of L||^2
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) col2 += __shfl_xor(col2, off);
    return n > 0 ? tr * col2 / n : 0.0;
}

template <typename T, int LP, int NC, bool GRAM>
__global__ __launch_bounds__(64 * W) void k_omp_scale(ScaleArgs a)
{
    constexpr int LPA = GRAM ? LP_GRAM : LP;
    __shared__ WaveLds<T, LPA> lds[W];
    __shared__ double lds64[W][KM * KM + 3 * KM];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * W + wv;
    if (b >= a.b) return;  // whole wavefront leaves together
    WaveLds<T, LPA> &w = lds[wv];
    const T *y = (const T *)a.y + b * (int64_t)a.y_stride;
    const int lp = GRAM ? a.lp : LP;

    // ---- measurement in the scale's coordinates -------------------------
    int rank_bound = 0;
    for (int t0 = 0; t0 < lp; t0 += 64) {
        const int t = t0 + lane;
        bool nz = false;
        if (t < lp) {
            T yh = 0, sq = 0;
            if (a.fold == kFold) {
                if (t < a.l) {
                    T cnt = 0, acc = 0;
                    const int j0 = a.blk_off[t], j1 = a.blk_off[t + 1];
                    for (int jj = j0; jj < j1; ++jj) {
                        const int j = a.blk_idx[jj];
                        const bool obs = a.mask ? a.mask[b * (int64_t)a.n + j] != 0 : true;
                        if (obs) { cnt += T(1); acc += y[j]; }
                    }
                    sq = sqrt(cnt);
                    yh = cnt > T(0) ? acc / sq : T(0);
                    nz = cnt > T(0);
                }
            } else {
                if (t < a.l) { yh = y[t]; sq = T(1); nz = true; }
            }
            w.yhat[t] = yh;
            w.sqw[t] = sq;
        }
        rank_bound += __popcll(__ballot(nz));
    }
    if (a.fold != kFold) rank_bound = a.m_dense;

    // ---- candidate set ---------------------------------------------------
    int nc;
    if (a.first) {
        nc = a.t;
    } else {
        const int kp = a.prev_kused[b];
        const int *ps = a.prev_sup + b * (int64_t)a.prev_stride;
        if (lane < kp) {
            const int pi = ps[lane];
            int rank = 0;
            for (int j = 0; j < kp; ++j) rank += ps[j] < pi;
            w.par[rank] = pi;
        }
        nc = kp * a.q;
    }
    int kreq = a.kvec ? a.kvec[b] : a.kuni;
    int K = kreq < nc ? kreq : nc;
    K = K < KM ? K : KM;
    K = K < a.sup_count ? K : a.sup_count;
    K = K > 0 ? K : 0;
    wave_sync();

    // ---- per-candidate state --------------------------------------------
    T v[GRAM ? 1 : NC][GRAM ? 1 : LP];
    T c[NC], e[NC], e0[NC], nu[NC];
    T u[NC][KM];
    int atom[NC];
    bool live[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const int ci = s * 64 + lane;
        live[s] = ci < nc;
        atom[s] = INT_MAX;
        if (live[s]) atom[s] = a.first ? ci : w.par[ci / a.q] * a.q + ci % a.q;
#pragma unroll
        for (int m = 0; m < KM; ++m) u[s][m] = T(0);
        T h = 0, ee = 0;
        if constexpr (!GRAM) {
            const T *src = (const T *)a.v + (int64_t)(live[s] ? atom[s] : 0) * LP;
#pragma unroll
            for (int j = 0; j < LP; ++j) {
                T x = live[s] ? src[j] : T(0);
                x *= w.sqw[j];
                v[s][j] = x;
                h += x * w.yhat[j];
                ee += x * x;
            }
        } else {
            if (live[s]) {
                const T *src = (const T *)a.v + (int64_t)atom[s] * lp;
                for (int j = 0; j < lp; ++j) {
                    T x = src[j] * w.sqw[j];
                    h += x * w.yhat[j];
                    ee += x * x;
                }
            }
        }
        c[s] = h;
        e[s] = ee;
        e0[s] = ee;
        nu[s] = sqrt(ee);
        if (!(ee > T(0))) live[s] = false;  // an effective column of zero is never picked
    }

    // ---- OMP iterations (Algorithm 1) -----------------------------------
    int n = 0;
    T lmax = 0, lmin = 0;
    for (int it = 0; it < K; ++it) {
        // proxy: |<a_i, r>| / ||a_i||, lowest index on ties
        T best = T(-1);
        int bidx = INT_MAX;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            if (live[s]) {
                const T sc = fabs(c[s]) / nu[s];
                if (sc > best) { best = sc; bidx = atom[s]; }
            }
        }
        wave_argmax(best, bidx);
        if (best < T(0)) break;  // candidates exhausted
        // the owning lane publishes its column, its u row and its scalars
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            if (live[s] && atom[s] == bidx) {
                if constexpr (!GRAM) {
#pragma unroll
                    for (int j = 0; j < LP; ++j) w.vk[j] = v[s][j];
                }
#pragma unroll
                for (int m = 0; m < KM; ++m) w.uk[m] = u[s][m];
                w.sc[0] = c[s];
                w.sc[1] = e[s];
                w.sc[2] = e0[s];
            }
        }
        wave_sync();
        const T ck = w.sc[0], ek = w.sc[1], e0k = w.sc[2];
        if (n >= rank_bound) break;                 // support already spans the space
        T lnn;
        if constexpr (sizeof(T) == 4) {
            // the pivot's own condition estimate: ratio of squared diagonals of L
            const T hi = n == 0 ? ek : (lmax * lmax > ek ? lmax * lmax : ek);
            const T lo = n == 0 ? ek : (lmin * lmin < ek ? lmin * lmin : ek);
            if (!(lo > T(0)) || hi > T(1e6) * lo) {
                // FP64 pivot: Cholesky of the FP64 Gram of Omega + {k}
                if (lane == 0) w.sup[n] = bidx;
                wave_sync();
                double *g64 = lds64[wv];
                double *h64 = g64 + KM * KM;
                double *dg = h64 + KM;
                gram64_chol<T, LPA>(w, a, w.sup, n + 1, lane, g64, h64, dg, false);
                const double piv = dg[KM + n], gkk = dg[n];
                if (!(piv > 1e-10 * gkk)) break;      // dependent in FP64 as well
                lnn = (T)sqrt(piv);
            } else {
                if (!(ek > dep_tol<T>() * e0k)) break;  // picked atom is dependent
                lnn = sqrt(ek);
            }
        } else {
            if (!(ek > dep_tol<T>() * e0k)) break;      // picked atom is dependent
            lnn = sqrt(ek);
        }
        const T inv = T(1) / lnn;
        const T zn = ck * inv;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            T g = 0;
            if constexpr (!GRAM) {
#pragma unroll
                for (int j = 0; j < LP; ++j) g += v[s][j] * w.vk[j];
            } else {
                if (atom[s] != INT_MAX) g = ((const T *)a.gram)[(int64_t)bidx * a.t + atom[s]];
            }
            T dot = 0;
#pragma unroll
            for (int m = 0; m < KM; ++m) dot += w.uk[m] * u[s][m];
            const T un = (g - dot) * inv;
#pragma unroll
            for (int m = 0; m < KM; ++m) u[s][m] = (m == n) ? un : u[s][m];
            c[s] -= un * zn;
            e[s] -= un * un;
            if (atom[s] == bidx) live[s] = false;
        }
        if (lane == 0) {
            w.sup[n] = bidx;
            w.z[n] = zn;
            for (int m = 0; m < n; ++m) w.lmat[n][m] = w.uk[m];
            w.lmat[n][n] = lnn;
        }
        lmax = n == 0 ? lnn : (lnn > lmax ? lnn : lmax);
        lmin = n == 0 ? lnn : (lnn < lmin ? lnn : lmin);
        ++n;
        wave_sync();
    }

    // ---- outputs ---------------------------------------------------------
    if (lane == 0) a.kused_out[b] = n;
    int *sup_out = a.sup_out + b * (int64_t)a.sup_stride;
    if (!a.last) {
        for (int i = lane; i < a.sup_count; i += 64) sup_out[i] = i < n ? w.sup[i] : -1;
        return;
    }
    // projection coefficients: L^T alpha = z
    if (lane == 0) {
        for (int i = n - 1; i >= 0; --i) {
            T s = w.z[i];
            for (int m = i + 1; m < n; ++m) s -= w.lmat[m][i] * w.alpha[m];
            w.alpha[i] = s / w.lmat[i][i];
        }
    }
    wave_sync();
    if constexpr (sizeof(T) == 4) {
        // FP64 back-substitution when FP32 normal equations would miss the
        // coefficient tolerance (their error grows like kappa(G) * 2^-24)
        if (n > 1 && cond_estimate<T, LPA>(w, n, lane) > 1e2) {
            double *g64 = lds64[wv];
            double *h64 = g64 + KM * KM;
            gram64_chol<T, LPA>(w, a, w.sup, n, lane, g64, h64, h64 + KM, true);
            if (lane == 0)
                for (int i = 0; i < n; ++i) w.alpha[i] = (T)h64[i];
            wave_sync();
        }
    }
    T *coef = (T *)a.coef_out + b * (int64_t)a.sup_stride;
    for (int i = lane; i < a.sup_count; i += 64) {
        sup_out[i] = i < n ? w.sup[i] : -1;
        coef[i] = i < n ? w.alpha[i] : T(0);
    }
    if (a.xhat) {
        const T *dh = (const T *)a.d_high;
        T *xh = (T *)a.xhat + b * (int64_t)a.n;
        for (int j = lane; j < a.n; j += 64) {
            T acc = 0;
            for (int i = 0; i < n; ++i) acc += w.alpha[i] * dh[(int64_t)w.sup[i] * a.n + j];
            xh[j] = acc;
        }
    }
}

template <typename T, int LP, int NC, bool GRAM>
cspd_status launch_one(const ScaleArgs &a, hipStream_t st)
{
    const unsigned grid = (unsigned)((a.b + W - 1) / W);
    char label[96];
    if (a.first && a.last)
        snprintf(label, sizeof(label), "omp_scale<%s,%s,lp%d,nc%d>:full", sizeof(T) == 8 ? "f64" : "f32",
                 GRAM ? "gram" : "vec", GRAM ? a.lp : LP, NC);
    else
        snprintf(label, sizeof(label), "omp_scale<%s,%s,lp%d,nc%d>:s%d", sizeof(T) == 8 ? "f64" : "f32",
                 GRAM ? "gram" : "vec", GRAM ? a.lp : LP, NC, a.scale);
    ProfileToken *tok = profile_begin(label, st);
    hipLaunchKernelGGL((k_omp_scale<T, LP, NC, GRAM>), dim3(grid), dim3(64 * W), 0, st, a);
    profile_end(tok, st);
    CSPD_HIP_CHECK(hipGetLastError());
    return CSPD_OK;
}

template <typename T>
cspd_status dispatch(const ScaleArgs &a, int max_cand, bool gram, hipStream_t st)
{
    const int ncs = (max_cand + 63) / 64;
    if (!gram) {
        switch (a.lp) {
            case 16: return ncs <= 1 ? launch_one<T, 16, 1, false>(a, st) : ncs <= 2 ? launch_one<T, 16, 2, false>(a, st) : CSPD_E_UNSUPPORTED;
            case 32: return ncs <= 1 ? launch_one<T, 32, 1, false>(a, st) : ncs <= 2 ? launch_one<T, 32, 2, false>(a, st) : CSPD_E_UNSUPPORTED;
            case 64: return ncs <= 1 ? launch_one<T, 64, 1, false>(a, st) : ncs <= 2 ? launch_one<T, 64, 2, false>(a, st) : CSPD_E_UNSUPPORTED;
            case 128: return ncs <= 1 ? launch_one<T, 128, 1, false>(a, st) : CSPD_E_UNSUPPORTED;
            default: return CSPD_E_UNSUPPORTED;
        }
    }
    if (a.lp > LP_GRAM) return CSPD_E_UNSUPPORTED;
    if (ncs <= 1) return launch_one<T, 0, 1, true>(a, st);
    if (ncs <= 2) return launch_one<T, 0, 2, true>(a, st);
    if (ncs <= 4) return launch_one<T, 0, 4, true>(a, st);
    if (ncs <= 8) return launch_one<T, 0, 8, true>(a, st);
    if (ncs <= 16) return launch_one<T, 0, 16, true>(a, st);
    return CSPD_E_UNSUPPORTED;
}

}  // namespace

// Whether a vec-mode kernel exists for this row length and candidate count.
bool scale_vec_fits(int lp, int max_cand)
{
    const int ncs = (max_cand + 63) / 64;
    return (lp == 16 || lp == 32 || lp == 64) ? ncs <= 2 : (lp == 128 ? ncs <= 1 : false);
}

cspd_status launch_scale(int dtype, const ScaleArgs &a, int max_cand, bool gram, hipStream_t st)
{
    if (a.b <= 0) return CSPD_OK;
    return dtype == CSPD_F64 ? dispatch<double>(a, max_cand, gram, st)
                             : dispatch<float>(a, max_cand, gram, st);
}

}  // namespace cspd
