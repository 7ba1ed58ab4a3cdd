// First scale of the cross-scale model on the matrix cores (problem (P_low)
// of Section III-C: every atom of D_0 is a candidate, and D_0 is shared by
// all patches).
//
// A wavefront owns 16 patches; patch j lives on lanes j, j + 16, j + 32 and
// j + 48, each of which holds a quarter of the patch's coordinates.  Each
// iteration of Algorithm 1 forms the proxy of every atom for the 16 patches
// at once,
//   C = D_0^T (s (.) r)      (atoms x patches; s = square-root fold weights),
// as 16 x 16 x 4 FP32 MFMA tiles whose A operand (the shared dictionary)
// stays in registers for the whole launch; a lane ends with the proxies of
// four atoms per tile for its own patch.  The support update is a per-patch
// modified Gram-Schmidt step on the patch's four lanes: the selected weighted
// atom is orthogonalised against the basis of the support so far and the
// residual loses its component along the new direction, so that
// r = (I - P_Omega) y-hat after every step, as the projection and residue
// steps of Algorithm 1 require.  Only the supports leave this kernel (a coarse
// scale's coefficients are not part of the output).
#include "omp_scale_impl.h"

namespace cspd {
namespace first_impl {

using scale_impl::swap_pair;
using scale_impl::swap_pair_i;

constexpr int W = 4;            // wavefronts per workgroup
constexpr int PW = 16;          // patches per wavefront
constexpr int NMAX = 64;        // fine samples staged per patch (fold plans)

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Sum of a value over the four lanes of a patch (lanes j + 16 q).
__device__ __forceinline__ float quad_sum(float v)
{
    float a, b;
    swap_pair<16>(v, a, b);
    v = a + b;
    swap_pair<32>(v, a, b);
    return a + b;
}

__device__ __forceinline__ double quad_sum(double v)
{
    double a, b;
    swap_pair<16>(v, a, b);
    v = a + b;
    swap_pair<32>(v, a, b);
    return a + b;
}

// Best (score, atom) over the four lanes of a patch: larger score, then the
// lower atom.
__device__ __forceinline__ void quad_argmax(float &s, int &i)
{
    float s0, s1;
    int i0, i1;
    swap_pair<16>(s, s0, s1);
    swap_pair_i<16>(i, i0, i1);
    scale_impl::argmax_merge(s0, i0, s1, i1, s, i);
    swap_pair<32>(s, s0, s1);
    swap_pair_i<32>(i, i0, i1);
    scale_impl::argmax_merge(s0, i0, s1, i1, s, i);
}

// LDS of one workgroup: the shared dictionary (padded rows), the block table
// of the fold, and per wavefront the staged measurements of its patches.
template <int L, int T>
struct FirstLds {
    float v[T][L + 1];
    int tab[NMAX + 1 + NMAX];
    float ys[W][PW][NMAX + 1];
    unsigned char ms[W][PW][NMAX + 4];
};

// FP64 Cholesky pivot of the Gram matrix of atoms ids[0..n1), weighted by the
// fold weights sw of this lane's coordinates (the four lanes of the patch
// each add their quarter).  Returns the last squared pivot and, in *gkk, the
// last diagonal entry.  For pivots far outside the range of the earlier ones.
template <int LQ, int KM>
__device__ __attribute__((noinline)) double pivot64(const float *v, int stride, const int *ids, int n1,
                                                  const float *sw, int qd, double *gkk)
{
    double g[KM + 1][KM + 1];
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int m = 0; m < LQ; ++m) {
                const double wt = (double)sw[m];
                s += ((double)v[ids[i] * stride + qd * LQ + m] * wt) *
                     ((double)v[ids[j] * stride + qd * LQ + m] * wt);
            }
            g[i][j] = quad_sum(s);
        }
    *gkk = g[n1 - 1][n1 - 1];
    double piv = 0.0;
    for (int j = 0; j < n1; ++j) {
        double d = g[j][j];
        for (int m = 0; m < j; ++m) d -= g[j][m] * g[j][m];
        piv = d;
        const double rj = d > 0.0 ? sqrt(d) : 0.0;
        for (int i = j + 1; i < n1; ++i) {
            double t = g[i][j];
            for (int m = 0; m < j; ++m) t -= g[i][m] * g[j][m];
            g[i][j] = rj > 0.0 ? t / rj : 0.0;
        }
    }
    return piv;
}

// LQ coordinates per lane (4 LQ per patch), NT tiles of 16 atoms, KM
// iterations at most.
template <int LQ, int NT, int KM>
// Four coordinates per lane and K <= 4: three wavefronts per SIMD (a few
// registers spill, outside the iterations' inner work)
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu((LQ == 4 && KM == 4) ? 3 : 1)))
void k_omp_first(ScaleArgs a)
{
    constexpr int L = 4 * LQ;
    constexpr int T = 16 * NT;
    static_assert(NT <= 8, "atom bits of a lane fit one word");
    __shared__ FirstLds<L, T> sh;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wavefront-uniform
    const int pj = lane & 15;           // patch within the wavefront
    const int qd = lane >> 4;           // coordinate quarter
    const int64_t first_patch = ((int64_t)blockIdx.x * W + wv) * PW;
    const int64_t b = first_patch + pj;
    const bool valid = b < a.b;
    const bool fold = a.fold == kFold;

    // ---- staging: every load is issued before the first LDS store (one
    // round trip to memory) --------------------------------------------------
    // workgroup: the dictionary, DV values per thread
    constexpr int DV = T * L / (64 * W);
    static_assert(T * L % (64 * W) == 0, "dictionary staging: whole passes of the workgroup");
    float dst[DV];
#pragma unroll
    for (int r = 0; r < DV; ++r) {
        const int i = threadIdx.x + r * 64 * W;
        const int t = i / L, j = i % L;
        dst[r] = (t < a.t && j < a.l) ? ((const float *)a.v)[(int64_t)t * a.lp + j] : 0.f;
    }
    // wavefront: its patches' samples, one row per patch, a lane per sample
    // (ny <= 64; each row coalesced)
    const int ny = fold ? a.n : a.l;
    const bool lin = lane < ny;
    const int jl = lin ? lane : 0;
    const bool has_mask = fold && a.mask;
    float yst[PW];
    unsigned char mst[PW];
#pragma unroll
    for (int p = 0; p < PW; ++p) {
        const int64_t row = first_patch + p < a.b ? first_patch + p : a.b - 1;
        yst[p] = ((const float *)a.y)[row * (int64_t)a.y_stride + jl];
        mst[p] = has_mask ? a.mask[row * (int64_t)a.n + jl] : (unsigned char)1;
    }
    // the fold's block table (at most 1 + 2 NMAX entries: one pass)
    const int ntab = fold ? a.l + 1 + a.n : 0;
    const int it = threadIdx.x;
    const int tabv = it < ntab ? (it <= a.l ? a.blk_off[it] : a.blk_idx[it - a.l - 1]) : 0;
#pragma unroll
    for (int r = 0; r < DV; ++r) {
        const int i = threadIdx.x + r * 64 * W;
        sh.v[i / L][i % L] = dst[r];
    }
    if (it < ntab) sh.tab[it] = tabv;
    if (lin) {
#pragma unroll
        for (int p = 0; p < PW; ++p) {
            sh.ys[wv][p][lane] = yst[p];
            sh.ms[wv][p][lane] = mst[p];
        }
    }
    __syncthreads();

    // ---- dictionary operand of the MFMA tiles (kept for the launch) -------
    // tile t, step m: lane -> atom 16 t + pj, coordinate qd LQ + m
    float dv[NT][LQ];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int m = 0; m < LQ; ++m) dv[t][m] = sh.v[16 * t + pj][qd * LQ + m];

    // ---- measurement in the scale's coordinates (this lane's quarter) -----
    float yh[LQ], sw[LQ];
    int nz = 0;
#pragma unroll
    for (int m = 0; m < LQ; ++m) {
        const int t = qd * LQ + m;
        float y_ = 0.f, s_ = 0.f;
        if (t < a.l) {
            if (fold) {
                float cnt = 0.f, acc = 0.f;
                const int j0 = sh.tab[t], j1 = sh.tab[t + 1];
                for (int jj = j0; jj < j1; ++jj) {
                    const int j = sh.tab[a.l + 1 + jj];
                    const bool obs = valid && sh.ms[wv][pj][j] != 0;
                    cnt += obs ? 1.f : 0.f;
                    acc += obs ? sh.ys[wv][pj][j] : 0.f;
                }
                s_ = scale_impl::fast_sqrt(cnt);
                y_ = cnt > 0.f ? acc * __builtin_amdgcn_rsqf(cnt) : 0.f;
                nz += cnt > 0.f;
            } else {
                s_ = 1.f;
                y_ = valid ? sh.ys[wv][pj][t] : 0.f;
            }
        }
        yh[m] = y_;
        sw[m] = s_;
    }
    const int rank_bound = fold ? (int)quad_sum((float)nz) : a.m_dense;

    // ---- inverse norms of the weighted atoms: (D_0 (.) D_0)^T s^2 ----------
    float inv_nu[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < LQ; ++m)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(dv[t][m] * dv[t][m], sw[m] * sw[m], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) inv_nu[t][r] = acc[r] > 0.f ? __builtin_amdgcn_rsqf(acc[r]) : -1.f;
    }

    int K = 0;
    if (valid) {
        K = a.kuni < a.t ? a.kuni : a.t;
        K = K < KM ? K : KM;
        K = K < a.sup_count ? K : a.sup_count;
        K = K > 0 ? K : 0;
    }
    // the wavefront runs the largest K of its patches
    const int kwave = __builtin_amdgcn_readfirstlane(scale_impl::group_max<64>(K));

    // ---- Algorithm 1 --------------------------------------------------------
    float rr[LQ];                        // residual, weighted coordinates
#pragma unroll
    for (int m = 0; m < LQ; ++m) rr[m] = yh[m];
    float qb[KM][LQ];                    // orthonormal basis of span(A_Omega)
    unsigned used = 0u;                  // bit 4 t + r: this lane's atom already chosen
    int sup[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) sup[i] = 0;
    int nsel = 0;
    bool active = K > 0;
    float pmax = 0.f, pmin = 0.f;        // range of the squared pivots
#pragma unroll
    for (int n = 0; n < KM; ++n) {
        if (n >= kwave) break;
        bool act = active && n < K;
        // proxy of every atom of this lane (slot 4 t + r is atom 16 t + 4 qd + r:
        // slots ascend with the atom index)
        float scs[4 * NT];
        int sid[4 * NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int m = 0; m < LQ; ++m)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(dv[t][m], sw[m] * rr[m], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool ok = inv_nu[t][r] > 0.f && !((used >> (4 * t + r)) & 1u);
                scs[4 * t + r] = ok ? fabsf(acc[r]) * inv_nu[t][r] : -1.f;
                sid[4 * t + r] = 4 * t + r;
            }
        }
        // best slot by a pairwise tree (depth log2(4 NT) instead of a chain):
        // the left slot of a pair is the lower atom, so '>' keeps it on ties
#pragma unroll
        for (int wd = 1; wd < 4 * NT; wd *= 2)
#pragma unroll
            for (int f = 0; f + wd < 4 * NT; f += 2 * wd) {
                const bool up = scs[f + wd] > scs[f];
                scs[f] = up ? scs[f + wd] : scs[f];
                sid[f] = up ? sid[f + wd] : sid[f];
            }
        float bsc = scs[0];
        int bidx = 16 * (sid[0] >> 2) + 4 * qd + (sid[0] & 3);
        quad_argmax(bsc, bidx);
        act = act && bsc >= 0.f && n < rank_bound;
        const int k = act ? bidx : 0;
        // the selected weighted atom on this lane's coordinates
        float ak[LQ];
        float nk = 0.f;
#pragma unroll
        for (int m = 0; m < LQ; ++m) {
            ak[m] = sh.v[k][qd * LQ + m] * sw[m];
            nk += ak[m] * ak[m];
        }
        nk = quad_sum(nk);
        // modified Gram-Schmidt against the basis so far
#pragma unroll
        for (int j = 0; j < KM; ++j) {
            if (j < n) {
                float pr = 0.f;
#pragma unroll
                for (int m = 0; m < LQ; ++m) pr += qb[j][m] * ak[m];
                pr = quad_sum(pr);
#pragma unroll
                for (int m = 0; m < LQ; ++m) ak[m] -= pr * qb[j][m];
            }
        }
        float rho2 = 0.f;
#pragma unroll
        for (int m = 0; m < LQ; ++m) rho2 += ak[m] * ak[m];
        rho2 = quad_sum(rho2);
        // the pivot's own condition estimate: a squared pivot far outside the
        // range of the earlier ones is decided in FP64
        const float hi = n == 0 ? rho2 : fmaxf(pmax, rho2);
        const float lo = n == 0 ? rho2 : fminf(pmin, rho2);
        const bool need64 = act && (!(lo > 0.f) || hi > 1e6f * lo);
        // dependent atom: its component outside span(A_Omega) is negligible
        if (act && !need64 && !(rho2 > 1e-5f * nk)) act = false;
        if (need64) {
            int ids[KM + 1];
            float swc[LQ];
#pragma unroll
            for (int i = 0; i < KM; ++i) ids[i] = sup[i];
            ids[n] = k;
#pragma unroll
            for (int m = 0; m < LQ; ++m) swc[m] = sw[m];
            double gkk = 0.0;
            const double piv = pivot64<LQ, KM>(&sh.v[0][0], L + 1, ids, n + 1, swc, qd, &gkk);
            if (!(piv > 1e-10 * gkk)) act = false;
            else if (!(rho2 > 0.f)) rho2 = (float)piv;
        }
        // new basis vector and the residual's component along it
        const float inv = act ? __builtin_amdgcn_rsqf(rho2) : 0.f;
        float zc = 0.f;
#pragma unroll
        for (int m = 0; m < LQ; ++m) {
            qb[n][m] = ak[m] * inv;
            zc += qb[n][m] * rr[m];
        }
        zc = quad_sum(zc);
#pragma unroll
        for (int m = 0; m < LQ; ++m) rr[m] -= zc * qb[n][m];
        if (act) {
            sup[n] = k;
            pmax = n == 0 ? rho2 : fmaxf(pmax, rho2);
            pmin = n == 0 ? rho2 : fminf(pmin, rho2);
            nsel = n + 1;
            // the lane whose rows hold the atom marks it
            if (((k >> 2) & 3) == qd) used |= 1u << (4 * (k >> 4) + (k & 3));
        }
        active = active && act;
    }

    // ---- outputs: supports and their sizes --------------------------------
    if (valid && qd == 0) {
        a.kused_out[b] = nsel;
        int *so = a.sup_out + b * (int64_t)a.sup_stride;
#pragma unroll
        for (int i = 0; i < KM; ++i)
            if (i < a.sup_count) so[i] = i < nsel ? sup[i] : -1;
        for (int i = KM; i < a.sup_count; ++i) so[i] = -1;
    }
}

template <int LQ, int NT, int KM>
cspd_status launch(const ScaleArgs &a, hipStream_t st)
{
    const int64_t waves = (a.b + PW - 1) / PW;
    const unsigned grid = (unsigned)((waves + W - 1) / W);
    char label[112];
    snprintf(label, sizeof(label), "omp_first_mfma<f32,l%d,t%d,k%d>:s%d", 4 * LQ, 16 * NT, KM, a.scale);
    launch_timed(label, k_omp_first<LQ, NT, KM>, dim3(grid), dim3(64 * W), 0u, st, a);
    CSPD_HIP_CHECK(hipGetLastError());
    return CSPD_OK;
}

}  // namespace first_impl

// The first scale of a cross-scale call on the matrix cores when it fits:
// FP32, a uniform sparsity of at most 8, a vector length of at most 16 with
// up to 128 atoms (or 32 with up to 64), and fold plans with at most 64 fine
// samples.  Returns CSPD_E_UNSUPPORTED otherwise (nothing is launched).
bool first_mfma_fits(int dtype, const ScaleArgs &a)
{
    using namespace first_impl;
    if (dtype != CSPD_F32 || !a.first || a.last || a.kvec) return false;
    if (a.fold == kFold && a.n > NMAX) return false;
    const int k = a.kuni < a.sup_count ? a.kuni : a.sup_count;
    if (k > 8) return false;
    return (a.l <= 16 && a.t <= 128) || (a.l <= 32 && a.t <= 64);
}

cspd_status launch_first_mfma(int dtype, const ScaleArgs &a, hipStream_t st)
{
    using namespace first_impl;
    if (!first_mfma_fits(dtype, a)) return CSPD_E_UNSUPPORTED;
    const int k = a.kuni < a.sup_count ? a.kuni : a.sup_count;
    if (a.b <= 0) return CSPD_OK;
    const bool k4 = k <= 4;
    if (a.l <= 16) {
        if (a.t <= 32) return k4 ? launch<4, 2, 4>(a, st) : launch<4, 2, 8>(a, st);
        if (a.t <= 64) return k4 ? launch<4, 4, 4>(a, st) : launch<4, 4, 8>(a, st);
        if (a.t <= 128) return k4 ? launch<4, 8, 4>(a, st) : launch<4, 8, 8>(a, st);
    } else if (a.l <= 32) {
        if (a.t <= 32) return k4 ? launch<8, 2, 4>(a, st) : launch<8, 2, 8>(a, st);
        if (a.t <= 64) return k4 ? launch<8, 4, 4>(a, st) : launch<8, 4, 8>(a, st);
    }
    return CSPD_E_UNSUPPORTED;
}

}  // namespace cspd
