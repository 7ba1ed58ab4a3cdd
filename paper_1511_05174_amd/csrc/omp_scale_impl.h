// Per-patch OMP over one scale of the cross-scale model (template body).
//
// A group of G = 64 / PPW lanes of one wavefront owns one patch (PPW patches
// per wavefront).  Lanes own candidate atoms: slot s of group lane l holds
// candidate s*G + l.  At scale 0 every atom of D_0 is a candidate (problem
// (P_low) of Section III-C); at finer scales the candidates are the child
// blocks f(Omega) of the previous scale's support (Section III-B, problem
// (P_high), Algorithm 2).
//
// Each OMP iteration (Algorithm 1: proxy, support merge, projection, residue)
// is carried in candidate coordinates with an incremental Cholesky factor L of
// the support's Gram matrix:
//   u_i = L^{-1} A_Omega^T a_i      row n of L is [u_k^T, sqrt(e_k)] when k joins
//   c_i = <a_i, r> = h_i - u_i^T z   z = L^{-1} A_Omega^T y
//   e_i = ||(I - P_Omega) a_i||^2 = ||a_i||^2 - ||u_i||^2
// so a step costs one Gram column <a_i, a_k> per candidate plus rank-1 updates
// of c, e and u; the residue is carried as its correlations with the
// candidates.  Group lane j also carries column j of L^{-1}, so that the
// coefficients alpha = L^{-T} z and a condition estimate of the Gram matrix
// come out lane-parallel at the end.
//
// Candidate vectors live in VGPRs (vec mode) or, for small dictionaries under
// a shared operator, the Gram column is read from the plan (gram mode).
// Cross-lane steps use DPP and the gfx950 permlane swaps; the selected atom's
// data reaches the group through one LDS broadcast per iteration.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>

#include "cspd_internal.h"

namespace cspd {
namespace scale_impl {

// Wavefronts per workgroup: one for the matrix-core Gram kernels (their
// wavefronts share nothing; measured faster than two, four or eight), the
// library's default for the others (one was 1.5x slower for the Gram-table
// kernel over 1,024 atoms).
template <bool MG>
constexpr int waves_per_block() { return MG ? 1 : kWavesPerBlock; }
constexpr int KX = kMaxK;        // FP64 rare-path table size
// Condition estimates tr(G) tr(G^{-1}) / n of the final support's Gram
// matrix above which the coefficients take one step of mixed-precision
// refinement, and above which they are re-solved in FP64 altogether.
constexpr double kRefineEst = 10.0;
constexpr double kBackSubEst = 1e4;
constexpr int LP_GRAM = 256;     // LDS row length for gram-mode kernels

// LDS exchange between lanes of one wavefront.  Every LDS record of these
// kernels is private to one wavefront, and a wavefront's LDS operations are
// performed in issue order, so wavefront-scope fences only have to keep the
// compiler from reordering; no wait for the writes is needed.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Square root and reciprocal of a pivot.  FP32 uses the hardware
// instructions (about 1 ulp; the coefficients' error is dominated by the
// conditioning of the support), FP64 the correctly rounded forms.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

template <typename T> __device__ __forceinline__ T dep_tol();
template <> __device__ __forceinline__ double dep_tol<double>() { return 1e-10; }
template <> __device__ __forceinline__ float dep_tol<float>() { return 1e-5f; }

// ---- cross-lane primitives (groups of 16, 32 or 64 lanes) -----------------
enum { DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E, DPP_ROW_HALF_MIRROR = 0x141, DPP_ROW_MIRROR = 0x140 };

// Row-local lane permutation.  Every lane of the wavefront is active where
// these are used, so no lane reads a disabled one; written as an update with
// a zero `old` so that the compiler folds it into the consuming instruction.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) { return __int_as_float(dpp_i<CTRL>(__float_as_int(v))); }

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The two values a lane sees across a 16-row pair (WIDTH 16) or a 32-lane
// half pair (WIDTH 32): its own row's and the partner row's.
template <int WIDTH>
__device__ __forceinline__ void swap_pair_i(int v, int &a, int &b)
{
    if constexpr (WIDTH == 16) {
        auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        a = r[0]; b = r[1];
    } else {
        auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        a = r[0]; b = r[1];
    }
}

template <int WIDTH>
__device__ __forceinline__ void swap_pair(float v, float &a, float &b)
{
    int x, y;
    swap_pair_i<WIDTH>(__float_as_int(v), x, y);
    a = __int_as_float(x); b = __int_as_float(y);
}

template <int WIDTH>
__device__ __forceinline__ void swap_pair(double v, double &a, double &b)
{
    const long long bits = __double_as_longlong(v);
    int l0, l1, h0, h1;
    swap_pair_i<WIDTH>((int)bits, l0, l1);
    swap_pair_i<WIDTH>((int)(bits >> 32), h0, h1);
    a = __longlong_as_double(((long long)h0 << 32) | (unsigned)l0);
    b = __longlong_as_double(((long long)h1 << 32) | (unsigned)l1);
}

// (score, index) pairs: larger score wins, equal scores go to the smaller
// index.  Written with bitwise operators so the compiler emits selects, not
// branches.
template <typename T>
__device__ __forceinline__ bool beats(T s1, int i1, T s0, int i0)
{
    return (s1 > s0) | ((s1 == s0) & (i1 < i0));
}

template <typename T, int CTRL>
__device__ __forceinline__ void argmax_step(T &s, int &i)
{
    const T os = dpp<CTRL>(s);
    const int oi = dpp_i<CTRL>(i);
    const bool take = beats(os, oi, s, i);
    s = take ? os : s;
    i = take ? oi : i;
}

template <typename T>
__device__ __forceinline__ void argmax_merge(T s0, int i0, T s1, int i1, T &s, int &i)
{
    const bool take1 = beats(s1, i1, s0, i0);
    s = take1 ? s1 : s0;
    i = take1 ? i1 : i0;
}

// Group-wide argmax with ties to the lowest index; every lane of the group
// ends with the result.  FP32 scores are non-negative (or -1 for "none"):
// one integer reduction over their bit patterns finds the largest score, a
// second one the lowest index among the lanes that hold it.
template <int G>
__device__ __forceinline__ int group_max(int k)
{
    k = max(k, dpp_i<DPP_QUAD_XOR1>(k));
    k = max(k, dpp_i<DPP_QUAD_XOR2>(k));
    k = max(k, dpp_i<DPP_ROW_HALF_MIRROR>(k));
    k = max(k, dpp_i<DPP_ROW_MIRROR>(k));
    if constexpr (G >= 32) {
        int x, y;
        swap_pair_i<16>(k, x, y);
        k = max(x, y);
    }
    if constexpr (G >= 64) {
        int x, y;
        swap_pair_i<32>(k, x, y);
        k = max(x, y);
    }
    return k;
}

template <int G>
__device__ __forceinline__ int group_min(int k)
{
    k = min(k, dpp_i<DPP_QUAD_XOR1>(k));
    k = min(k, dpp_i<DPP_QUAD_XOR2>(k));
    k = min(k, dpp_i<DPP_ROW_HALF_MIRROR>(k));
    k = min(k, dpp_i<DPP_ROW_MIRROR>(k));
    if constexpr (G >= 32) {
        int x, y;
        swap_pair_i<16>(k, x, y);
        k = min(x, y);
    }
    if constexpr (G >= 64) {
        int x, y;
        swap_pair_i<32>(k, x, y);
        k = min(x, y);
    }
    return k;
}

template <int G>
__device__ __forceinline__ void group_argmax(float &s, int &i)
{
    // bit patterns of non-negative floats order like the floats; -1 is
    // negative as an integer
    const int sb = __float_as_int(s);
    const int mb = group_max<G>(sb);
    i = group_min<G>((sb == mb && mb >= 0) ? i : INT_MAX);
    s = __int_as_float(mb);
}

template <int G, typename T>
__device__ __forceinline__ void group_argmax(T &s, int &i)
{
    argmax_step<T, DPP_QUAD_XOR1>(s, i);
    argmax_step<T, DPP_QUAD_XOR2>(s, i);
    argmax_step<T, DPP_ROW_HALF_MIRROR>(s, i);
    argmax_step<T, DPP_ROW_MIRROR>(s, i);
    if constexpr (G >= 32) {
        T s0, s1;
        int i0, i1;
        swap_pair<16>(s, s0, s1);
        swap_pair_i<16>(i, i0, i1);
        argmax_merge(s0, i0, s1, i1, s, i);
    }
    if constexpr (G >= 64) {
        T s0, s1;
        int i0, i1;
        swap_pair<32>(s, s0, s1);
        swap_pair_i<32>(i, i0, i1);
        argmax_merge(s0, i0, s1, i1, s, i);
    }
}

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v)
{
    v += dpp<DPP_QUAD_XOR1>(v);
    v += dpp<DPP_QUAD_XOR2>(v);
    v += dpp<DPP_ROW_HALF_MIRROR>(v);
    v += dpp<DPP_ROW_MIRROR>(v);
    if constexpr (G >= 32) {
        T a, b;
        swap_pair<16>(v, a, b);
        v = a + b;
    }
    if constexpr (G >= 64) {
        T a, b;
        swap_pair<32>(v, a, b);
        v = a + b;
    }
    return v;
}

// The lanes of a 16-row pair (WIDTH 16) or of two 32-lane halves (WIDTH 32)
// exchange a (lower row / half) and b (upper): lane r of the lower one ends
// with (its a, the partner's a), of the upper one with (the partner's b, its
// b) -- so lo + hi sums a over the pair in the lower and b in the upper.
template <int WIDTH>
__device__ __forceinline__ void split_pair(double a, double b, double &lo, double &hi)
{
    const long long ba = __double_as_longlong(a), bb = __double_as_longlong(b);
    int l0, l1, h0, h1;
    if constexpr (WIDTH == 16) {
        auto rl = __builtin_amdgcn_permlane16_swap((int)ba, (int)bb, false, false);
        auto rh = __builtin_amdgcn_permlane16_swap((int)(ba >> 32), (int)(bb >> 32), false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    } else {
        auto rl = __builtin_amdgcn_permlane32_swap((int)ba, (int)bb, false, false);
        auto rh = __builtin_amdgcn_permlane32_swap((int)(ba >> 32), (int)(bb >> 32), false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    }
    lo = __longlong_as_double(((long long)h0 << 32) | (unsigned)l0);
    hi = __longlong_as_double(((long long)h1 << 32) | (unsigned)l1);
}

typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

// ci / q for a candidate index ci < 2^16 (the parent slot of child ci): one
// high multiply by the plan's ceil(2^32 / q), exact while q < 2^16
__device__ __forceinline__ int child_parent(int ci, const ScaleArgs &a)
{
    return a.q == 1 ? ci : (int)__umulhi((unsigned)ci, a.qmagic);
}

// Low parts of a two-term FP16 split: fp16(x - h) for the pair x with high
// parts h = fp16(x).  x - h is exact in FP32; v_fma_mix_f32 forms it from the
// packed FP16 h directly (h * -1 + x), one instruction per element.
__device__ __forceinline__ half2v split_lo(float2v x, half2v h)
{
    float r0, r1;
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r0) : "v"(h), "v"(x[0]));
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r1) : "v"(h), "v"(x[1]));
    const float2v r = {r0, r1};
    return __builtin_convertvector(r, half2v);
}

// Sums over a group of G = 32 or 64 lanes of KM per-lane values, sum i
// returned (as FP32) to lane i of the group (i < KM; other lanes get one of
// them).  Reduce-scatter: each exchange across 32-lane halves and across
// 16-lane rows splits the values between the partners, so the rows then
// sum only KM / 2 (G 32) or KM / 4 (G 64) values; one permute delivers them.
template <int G, int KM>
__device__ __forceinline__ float sums_to_lanes(const double (&v)[KM], int lane)
{
    static_assert((G == 32 || G == 64) && KM % (G / 16) == 0, "group of 32 or 64 lanes");
    constexpr int K1 = G == 64 ? KM / 2 : KM;   // after the step across halves
    constexpr int K2 = K1 / 2;                  // after the step across rows
    double a1[K1];
    if constexpr (G == 64) {
#pragma unroll
        for (int j = 0; j < K1; ++j) {
            double lo, hi;
            split_pair<32>(v[j], v[K1 + j], lo, hi);
            a1[j] = lo + hi;              // half h holds sums h K1 + j
        }
    } else {
#pragma unroll
        for (int j = 0; j < K1; ++j) a1[j] = v[j];
    }
    float a2[K2];
#pragma unroll
    for (int j = 0; j < K2; ++j) {
        double lo, hi;
        split_pair<16>(a1[j], a1[K2 + j], lo, hi);
        a2[j] = (float)group_sum<16>(lo + hi);   // row r (of its half) holds r K2 + j
    }
    // sum i lives on every lane q of row (i / K2) % 2 of half i / K1 as entry
    // i % K2; lane q offers entry q % K2 (K2 divides 16)
    const int q = lane & 15;
    float sel = a2[0];
#pragma unroll
    for (int j = 1; j < K2; ++j) sel = (q % K2) == j ? a2[j] : sel;
    const int i = (lane % G) < KM ? lane % G : 0;
    const int src = (lane / G) * G + (i / K1) * 32 + ((i / K2) & 1) * 16 + q;
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src * 4, __float_as_int(sel)));
}

template <int G>
__device__ __forceinline__ int group_count(bool pred, int lane)
{
    const unsigned long long m = __ballot(pred);
    if constexpr (G == 64) return __popcll(m);
    const int g = lane / G;
    return __popcll((m >> (g * G)) & ((1ull << G) - 1ull));
}

// ---- LDS layout: one record per patch group --------------------------------
template <typename T, int LPA, int KM, int PSN = 1>
struct alignas(16) GroupLds {
    // pre-split kernels: the FP16 split of t y-hat (high and low parts of
    // each coordinate pair) and each pair's observation pattern
    uint32_t ysh[PSN];
    uint32_t ysl[PSN];
    uint32_t mpat[PSN];
    alignas(16) T yhat[LPA];
    T sqw[LPA];
    T vk[LPA];
    T uk[KM];
    T alpha[KX];
    T sc[4];
    int sup[KX];
};

// FP64 Gram matrix and right-hand side of atoms ids[0..n-1] of one group,
// accumulated in FP64 from the stored vectors (all 64 lanes split the dot
// products), then on lane 0 an FP64 Cholesky in place (pivots kept in
// piv[0..n)) and, when `solve`, the two triangular solves (solution in h64).
// Arguments are passed by value: taking the address of the kernel's argument
// record would move it to scratch memory for the whole kernel.
template <typename T>
__device__ __attribute__((noinline)) void gram64_chol(const T *v, int lp, int l, const T *sqw,
                                                      const T *yhat, const int *ids, int n, int lane,
                                                      double *g64, double *h64, double *piv,
                                                      double *gdiag, bool solve)
{
    const int np = n * (n + 1) / 2;
    for (int pidx = lane; pidx < np + n; pidx += 64) {
        double s = 0.0;
        if (pidx < np) {
            int i = 0, rem = pidx;
            while (rem > i) { rem -= i + 1; ++i; }
            const int j = rem;  // j <= i
            const T *vi = v + (int64_t)ids[i] * lp;
            const T *vj = v + (int64_t)ids[j] * lp;
            for (int t = 0; t < l; ++t) {
                const double wt = (double)sqw[t];
                s += ((double)vi[t] * wt) * ((double)vj[t] * wt);
            }
            g64[i * KX + j] = s;
            g64[j * KX + i] = s;
        } else {
            const int i = pidx - np;
            const T *vi = v + (int64_t)ids[i] * lp;
            for (int t = 0; t < l; ++t) s += (double)vi[t] * (double)sqw[t] * (double)yhat[t];
            h64[i] = s;
        }
    }
    wave_sync();
    if (lane == 0) {
        for (int j = 0; j < n; ++j) gdiag[j] = g64[j * KX + j];
        for (int j = 0; j < n; ++j) {
            double d = g64[j * KX + j];
            for (int k = 0; k < j; ++k) d -= g64[j * KX + k] * g64[j * KX + k];
            piv[j] = d;
            const double r = d > 0.0 ? sqrt(d) : 0.0;
            for (int i = j + 1; i < n; ++i) {
                double t = g64[i * KX + j];
                for (int k = 0; k < j; ++k) t -= g64[i * KX + k] * g64[j * KX + k];
                g64[i * KX + j] = r > 0.0 ? t / r : 0.0;
            }
            g64[j * KX + j] = r;
        }
        if (solve) {
            for (int i = 0; i < n; ++i) {
                double t = h64[i];
                for (int k = 0; k < i; ++k) t -= g64[i * KX + k] * h64[k];
                h64[i] = g64[i * KX + i] > 0.0 ? t / g64[i * KX + i] : 0.0;
            }
            for (int i = n - 1; i >= 0; --i) {
                double t = h64[i];
                for (int k = i + 1; k < n; ++k) t -= g64[k * KX + i] * h64[k];
                h64[i] = g64[i * KX + i] > 0.0 ? t / g64[i * KX + i] : 0.0;
            }
        }
    }
    wave_sync();
}

template <typename T, int LP, int NC, int PPW, int KM, bool GRAM, bool MG, bool PS>
__global__ __launch_bounds__(64 * waves_per_block<MG>())
__attribute__((amdgpu_waves_per_eu((MG && PPW == 2 && LP <= 64 && KM <= 8) ? 4 : 1)))
void k_omp_scale(ScaleArgs a)
{
    constexpr int W = waves_per_block<MG>();
    static_assert(!MG || (sizeof(T) == 4 && NC == 1 && (PPW == 1 || PPW == 2) && !GRAM && LP >= 16 && LP <= 128),
                  "matrix-core Gram: FP32, one slot, one or two patches per wavefront");
    static_assert(!PS || MG, "pre-split candidates feed the matrix-core Gram");
    constexpr int PSN = PS ? LP / 2 : 1;
    constexpr int G = 64 / PPW;
    constexpr int LPA = GRAM ? LP_GRAM : LP;
    constexpr int VL = (GRAM || MG) ? 1 : LP;   // per-slot vector registers
    constexpr int LH = MG ? LP / 2 : 1;         // coordinates per lane and patch (matrix-core Gram)
    // 32 x 32 Gram blocks kept per wavefront: two patches, or one patch's
    // (0,0), (0,1) and (1,1) blocks; (1,0) is the transpose of (0,1)
    constexpr int NGM = (MG && PPW == 1) ? 3 : 2;
    constexpr bool G01T = MG && PPW == 1;       // (0,1) block also in LDS, column-major
    constexpr bool F16G = MG;                   // Gram from a split into FP16 products
    constexpr int G01S = 36;                    // its column stride (16-byte rows, banks spread)
    __shared__ GroupLds<T, LPA, KM, PSN> lds[W * PPW];
    __shared__ __attribute__((aligned(16))) float g01_lds[G01T ? W : 1][G01T ? 32 * G01S : 1];
    __shared__ __attribute__((aligned(16))) double lds64[W][KX * KX + 4 * KX];
    extern __shared__ double dyn_lds[];     // block-fold staging (fold_lds_bytes)
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int gi = lane / G;
    const int gl = lane % G;
    const int hh = lane >> 5;   // lane half (matrix-core Gram)
    const int64_t wave_first = ((int64_t)blockIdx.x * W + wv) * PPW;
    if (wave_first >= a.b) return;          // the whole wavefront leaves together
    const int64_t b = wave_first + gi;
    const bool valid = b < a.b;
    const int64_t bb = valid ? b : wave_first;   // a row that exists, for loads
    GroupLds<T, LPA, KM, PSN> &w = lds[wv * PPW + gi];
    const T *y = (const T *)a.y + bb * (int64_t)a.y_stride;
    // operator of the patch (plans with several): the slice of the candidate
    // vectors it reads; a phase out of range leaves the patch unsolved
    int ph = 0;
    bool phok = true;
    if (a.phase) {
        ph = a.phase[bb];
        phok = ph >= 0 && ph < a.n_phases;
        ph = phok ? ph : 0;
    }
    const T *vph = (const T *)a.v + (int64_t)ph * a.phase_stride;
    const int lp = GRAM ? a.lp : LP;

    // Every load of the prologue is issued into registers before any result
    // is used (one round trip to memory); the candidate vectors follow once
    // the candidate set is known.
    // ---- candidate set ---------------------------------------------------
    // At the first scale every atom is a candidate; at a finer scale the
    // candidates are the child blocks of the previous support, in the order
    // of that support (the order only places candidates on lanes: ties in
    // the proxy go to the lowest atom index).  Each lane then requests its
    // candidate vectors at once.
    T v[NC][VL];
    T c[NC], e[NC], e0[NC], nu[NC];
    T u[NC][KM];
    int atom[NC];
    bool live[NC];
    const T *src[NC];
    // Matrix-core Gram: with two patches per wavefront lane l holds candidate
    // l % 32 of both patches; with one patch (up to 64 candidates) it holds
    // candidates l % 32 and 32 + l % 32 (blocks 0 and 1).  Either way it holds
    // coordinates [(l / 32) LH, (l / 32 + 1) LH) of each (the MFMA's two k
    // rows split the coordinates in halves).
    // Long vectors go through the matrix cores in chunks of MCH coordinates
    // (loaded chunk by chunk), so that few registers hold them at a time.
    constexpr int MCH = (MG && (PPW == 1 || LH >= 64)) ? (PPW == 1 && LH >= 64 ? 8 : 16) : LH;
    T vm[MG ? 2 : 1][MCH];
    T vn[MG && MCH < LH ? 2 : 1][MCH < LH ? MCH : 1];   // next chunk, in flight
    const T *msrc[2] = {nullptr, nullptr};
    bool livep[2] = {false, false};
    int nc = 0;
    auto candidates = [&](int ncand, int pvv) {
        nc = ncand;
        if constexpr (MG) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                // two patches: slot p is patch p's candidate gl; one patch:
                // slot p is candidate 32 p + gl % 32
                const int ncp = __builtin_amdgcn_readlane(ncand, PPW == 2 ? p * 32 : 0);
                const int ci = PPW == 2 ? gl : 32 * p + (lane & 31);
                livep[p] = ci < ncp;
                int at = ci;
                if (!a.first) {
                    const int pj = livep[p] ? child_parent(ci, a) : 0;
                    const int pi = __shfl(pvv, (PPW == 2 ? p * 32 : 0) + pj, 64);
                    at = pi * a.q + (ci - pj * a.q);
                }
                // pre-split rows hold, per 8 coordinates, the four high-part
                // pairs then the four low-part pairs: LP 32-bit words per atom,
                // read exactly like the FP32 rows (bits only)
                const int php = PPW == 2 ? __builtin_amdgcn_readlane(ph, p * 32) : ph;
                msrc[p] = (const T *)(PS ? a.vsplit : a.v) + (int64_t)php * a.phase_stride +
                          (int64_t)(livep[p] ? at : 0) * LP + hh * LH;
                if constexpr (MCH == LH) {
#pragma unroll
                    for (int j = 0; j < LH; j += 4) {
                        const float4 q = *reinterpret_cast<const float4 *>(msrc[p] + j);
                        vm[p][j] = q.x; vm[p][j + 1] = q.y; vm[p][j + 2] = q.z; vm[p][j + 3] = q.w;
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int ci = s * G + gl;
            live[s] = ci < nc;
            int at = ci;
            if (!a.first) {
                // parent ci / q of the previous support, from the lane that loaded it
                const int pj = live[s] ? child_parent(ci, a) : 0;
                const int pi = __shfl(pvv, pj, G);
                at = pi * a.q + (ci - pj * a.q);
            }
            atom[s] = live[s] ? at : INT_MAX;
            src[s] = vph + (int64_t)(live[s] ? at : 0) * (GRAM ? lp : LP);
        }
        if constexpr (!GRAM && !MG) {
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                if constexpr (sizeof(T) == 4) {
#pragma unroll
                    for (int j = 0; j < LP; j += 4) {
                        const float4 q = *reinterpret_cast<const float4 *>(src[s] + j);
                        v[s][j] = q.x; v[s][j + 1] = q.y; v[s][j + 2] = q.z; v[s][j + 3] = q.w;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < LP; j += 2) {
                        const double2 q = *reinterpret_cast<const double2 *>(src[s] + j);
                        v[s][j] = q.x; v[s][j + 1] = q.y;
                    }
                }
            }
        }
    };
    if (a.first) candidates(valid ? a.t : 0, -1);   // needs no load

    // ---- previous support and sparsity -----------------------------------
    int kp = 0, pv = -1;
    if (!a.first) {
        kp = a.prev_kused[bb];
        if (a.prev_count > 0) {   // entries at or past prev_count are masked where used
            const int gc = gl < a.prev_count ? gl : 0;
            pv = a.prev_sup[bb * (int64_t)a.prev_stride + gc];
        }
    }
    const int kreq = a.kvec ? a.kvec[bb] : a.kuni;

    // ---- measurement samples (and the fold's block table) ----------------
    // Without blocks a lane reads the samples of its own coordinates (at most
    // lp of them); blocks stage all n samples through LDS further down.
    constexpr int NJ = GRAM ? 256 / G : (LP + G - 1) / G;
    const bool fold = a.fold == kFold;
    const bool blocks = fold && !a.blk_ident;
    const int ny = blocks ? 0 : a.l;       // samples of y read here
    const uint8_t *mrow = (fold && a.mask) ? a.mask + bb * (int64_t)a.n : nullptr;
    T yr[NJ];
    int mr[NJ];
#pragma unroll
    for (int r = 0; r < NJ; ++r) {
        yr[r] = T(0);
        mr[r] = 0;
        if (r * G < ny) {
            const int j = r * G + gl;
            const int jc = j < ny ? j : 0;
            yr[r] = y[jc];
            mr[r] = mrow ? (int)mrow[jc] : 1;
        }
    }

    if (!a.first) candidates(valid ? kp * a.q : 0, pv);

    // ---- measurement in the scale's coordinates -------------------------
    int rank_bound = 0;
    if (!fold) {
#pragma unroll
        for (int r = 0; r < NJ; ++r) {
            const int t = r * G + gl;
            if (r * G < lp && t < lp) {
                w.yhat[t] = (valid && t < a.l) ? yr[r] : T(0);
                w.sqw[t] = T(1);
            }
        }
        rank_bound = a.m_dense;
    } else if (!blocks) {
        // coordinate t is fine sample t: weight 1 if observed, else 0
#pragma unroll
        for (int r = 0; r < NJ; ++r) {
            if (r * G < lp) {
                const int t = r * G + gl;
                const bool obs = valid && t < a.l && mr[r] != 0;
                if (t < lp) {
                    w.yhat[t] = obs ? yr[r] : T(0);
                    w.sqw[t] = obs ? T(1) : T(0);
                }
                rank_bound += group_count<G>(obs, lane);
            }
        }
    } else {
        // blocks of several fine samples: stage the patch's observed samples
        // and the block table in LDS, then each lane folds its coordinates
        T *ys = (T *)dyn_lds + (wv * PPW + gi) * 2 * a.n;
        T *ms = ys + a.n;
        int *bo = (int *)((T *)dyn_lds + W * PPW * 2 * a.n) + wv * (a.l + 1 + a.n);
        int *bi = bo + a.l + 1;
        const int ntab = a.l + 1 + a.n;
#pragma unroll 4
        for (int i = lane; i < ntab; i += 64) bo[i] = i <= a.l ? a.blk_off[i] : a.blk_idx[i - a.l - 1];
#pragma unroll 4
        for (int j = gl; j < a.n; j += G) {
            const T yv = y[j];
            const int mk = mrow ? (int)mrow[j] : 1;
            const bool obs = valid && mk != 0;
            ys[j] = obs ? yv : T(0);
            ms[j] = obs ? T(1) : T(0);
        }
        wave_sync();
        for (int t0 = 0; t0 < lp; t0 += G) {
            const int t = t0 + gl;
            bool nz = false;
            if (t < lp) {
                T yh = 0, sq = 0;
                if (t < a.l) {
                    T cnt = 0, acc = 0;
                    const int j0 = bo[t], j1 = bo[t + 1];
                    for (int jj = j0; jj < j1; ++jj) {
                        const int j = bi[jj];
                        cnt += ms[j];
                        acc += ys[j];
                    }
                    sq = sqrt(cnt);
                    yh = cnt > T(0) ? acc / sq : T(0);
                    nz = cnt > T(0);
                }
                w.yhat[t] = yh;
                w.sqw[t] = sq;
            }
            rank_bound += group_count<G>(nz, lane);
        }
    }

    // Pre-split kernels: the measurement is split like the candidates, after
    // scaling by a power of two t (per patch) that brings its largest entry to
    // at most 2^14; correlations then come out scaled by t (and by the plan's
    // split scale s), which changes no comparison (t and s are powers of two).
    T ysc = T(1);
    if constexpr (PS) {
        wave_sync();
        T ym = T(0);
#pragma unroll
        for (int pi = gl; pi < LP / 2; pi += G) {
            const float2 yv = *reinterpret_cast<const float2 *>(&w.yhat[2 * pi]);
            ym = fmaxf(ym, fmaxf(fabsf(yv.x), fabsf(yv.y)));
        }
        // bit patterns of non-negative floats order like the floats
        const T ymax = __int_as_float(group_max<G>(__float_as_int(ym)));
        int ex = 0;
        (void)frexpf(ymax, &ex);             // ymax = m 2^ex, m in [0.5, 1)
        ex = ex < -40 ? -40 : (ex > 40 ? 40 : ex);
        ysc = ymax > T(0) ? ldexpf(1.f, 14 - ex) : T(1);
#pragma unroll
        for (int pi = gl; pi < LP / 2; pi += G) {
            const float2 yv = *reinterpret_cast<const float2 *>(&w.yhat[2 * pi]);
            const float2 sq = *reinterpret_cast<const float2 *>(&w.sqw[2 * pi]);
            const float2v xp = {yv.x * ysc, yv.y * ysc};
            const half2v hp = __builtin_convertvector(xp, half2v);
            const half2v lo = split_lo(xp, hp);
            w.ysh[pi] = __builtin_bit_cast(uint32_t, hp);
            w.ysl[pi] = __builtin_bit_cast(uint32_t, lo);
            w.mpat[pi] = (sq.x != T(0) ? 0x0000FFFFu : 0u) | (sq.y != T(0) ? 0xFFFF0000u : 0u);
        }
    }

    int K = 0;
    if (valid && phok) {
        K = kreq < nc ? kreq : nc;
        K = K < KM ? K : KM;
        K = K < a.sup_count ? K : a.sup_count;
        K = K > 0 ? K : 0;
    }
    // iterations the wavefront runs: the largest K of its groups
    int kwave = 0;
#pragma unroll
    for (int g = 0; g < PPW; ++g) {
        const int kg = __builtin_amdgcn_readlane(K, g * G);
        kwave = kg > kwave ? kg : kwave;
    }

    // ---- per-candidate state --------------------------------------------
    // The published u row starts at zero: a pick writes only the entries
    // filled so far, and a group that has stopped keeps reading entries no
    // pick wrote (times zero, which must not meet stale bits).
    if (gl < KM) w.uk[gl] = T(0);
    wave_sync();
#pragma unroll
    for (int s = 0; s < NC; ++s)
#pragma unroll
        for (int m = 0; m < KM; ++m) u[s][m] = T(0);
    T h[NC], ee[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) { h[s] = T(0); ee[s] = T(0); }
    typedef float gram_t __attribute__((ext_vector_type(16)));
    typedef _Float16 half8 __attribute__((ext_vector_type(8)));
    gram_t gm[NGM];
    if constexpr (MG) {
        // weighted candidates, their correlations with y-hat and squared norms
        // (each lane sums its half of the coordinates, the halves are added)
        // Gram matrices on the matrix cores: lane l ends with column l % 32,
        // rows 8 (r / 4) + 4 (l / 32) + r % 4 of each 32 x 32 block.  Two
        // patches: block p is patch p's Gram matrix.  One patch: blocks 0, 1
        // and 2 hold the products of candidate blocks (0,0), (0,1), (1,1)
        // (rows from the first block named, columns from the second).
        T hs[2] = {T(0), T(0)}, es[2] = {T(0), T(0)};
        T hs2[2] = {T(0), T(0)};   // pre-split: the two cross terms of the correlations
#pragma unroll
        for (int p = 0; p < NGM; ++p)
#pragma unroll
            for (int r = 0; r < 16; ++r) gm[p][r] = 0.f;
        // chunk c + 1 is requested before chunk c is used
        auto load_chunk = [&](int c0, T (&dst)[2][MCH < LH ? MCH : 1]) {
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int j = 0; j < MCH; j += 4) {
                    const float4 q = *reinterpret_cast<const float4 *>(msrc[p] + c0 + j);
                    dst[p][j] = q.x; dst[p][j + 1] = q.y; dst[p][j + 2] = q.z; dst[p][j + 3] = q.w;
                }
        };
        if constexpr (MCH < LH) load_chunk(0, vn);
#pragma unroll
        for (int c0 = 0; c0 < LH; c0 += MCH) {
            if constexpr (MCH < LH) {
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int j = 0; j < MCH; ++j) vm[p][j] = vn[p][j];
                if (c0 + MCH < LH) load_chunk(c0 + MCH, vn);
            }
#pragma unroll
            for (int p = 0; p < 2 && !PS; ++p) {
                const GroupLds<T, LPA, KM, PSN> &wp = lds[wv * PPW + (PPW == 2 ? p : 0)];
#pragma unroll
                for (int j = 0; j < MCH; ++j) {
                    const T sw = wp.sqw[hh * LH + c0 + j], yh = wp.yhat[hh * LH + c0 + j];
                    // split Gram: candidates scaled by a power of two (exact), see
                    // below.  With two patches a dead slot keeps atom 0's vector:
                    // its Gram row and column, h and e are never read (score -1)
                    const T xv = vm[p][j] * (F16G ? sw * a.gsplit : sw);
                    const T x = (PPW == 2 || livep[p]) ? xv : T(0);
                    vm[p][j] = x;
                    hs[p] += x * yh;
                    es[p] += x * x;
                }
            }
            if constexpr (PS) {
                // Pre-split candidates (plan time: s x = h + l, both FP16):
                // an unobserved coordinate clears its halves with the pair's
                // pattern (exact: the mask only selects), the correlations
                // with t y-hat = yh + yl come from packed FP16 dot products
                // with FP32 accumulation (h yh + h yl + l yh; l yl is below
                // FP32 rounding), and the Gram matrix from the same three
                // split products on the matrix cores as below.
                typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
                for (int c = 0; c < MCH; c += 8) {
                    half8 hv[2], lv[2];
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const GroupLds<T, LPA, KM, PSN> &wp = lds[wv * PPW + (PPW == 2 ? p : 0)];
                        const int pi = (hh * LH + c0 + c) / 2;
                        u32x4 pat = *reinterpret_cast<const u32x4 *>(&wp.mpat[pi]);
                        const u32x4 yh = *reinterpret_cast<const u32x4 *>(&wp.ysh[pi]);
                        const u32x4 yl = *reinterpret_cast<const u32x4 *>(&wp.ysl[pi]);
                        if constexpr (PPW == 1) {
                            const uint32_t keep = livep[p] ? 0xFFFFFFFFu : 0u;   // dead slots read as zero
                            pat &= keep;
                        }
                        // (vector elements are copied to scalars before a bit cast:
                        // a bit cast of an element reference reads element 0)
                        uint32_t mh[4], ml[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const uint32_t pe = pat[e], yhe = yh[e], yle = yl[e];
                            mh[e] = __float_as_uint(vm[p][c + e]) & pe;
                            ml[e] = __float_as_uint(vm[p][c + 4 + e]) & pe;
                            const half2v h2 = __builtin_bit_cast(half2v, mh[e]);
                            const half2v l2 = __builtin_bit_cast(half2v, ml[e]);
                            const half2v y2h = __builtin_bit_cast(half2v, yhe);
                            const half2v y2l = __builtin_bit_cast(half2v, yle);
                            hs[p] = __builtin_amdgcn_fdot2(h2, y2h, hs[p], false);
                            hs2[p] = __builtin_amdgcn_fdot2(h2, y2l, hs2[p], false);
                            hs2[p] = __builtin_amdgcn_fdot2(l2, y2h, hs2[p], false);
                        }
                        const u32x4 mhv = {mh[0], mh[1], mh[2], mh[3]};
                        const u32x4 mlv = {ml[0], ml[1], ml[2], ml[3]};
                        hv[p] = __builtin_bit_cast(half8, mhv);
                        lv[p] = __builtin_bit_cast(half8, mlv);
                    }
                    if constexpr (PPW == 1) {
                        gm[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[0], hv[0], gm[0], 0, 0, 0);
                        gm[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[0], lv[0], gm[0], 0, 0, 0);
                        gm[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lv[0], hv[0], gm[0], 0, 0, 0);
                        gm[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[0], hv[1], gm[1], 0, 0, 0);
                        gm[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[0], lv[1], gm[1], 0, 0, 0);
                        gm[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lv[0], hv[1], gm[1], 0, 0, 0);
                        gm[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[1], hv[1], gm[2], 0, 0, 0);
                        gm[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[1], lv[1], gm[2], 0, 0, 0);
                        gm[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lv[1], hv[1], gm[2], 0, 0, 0);
                    } else {
#pragma unroll
                        for (int p = 0; p < 2; ++p) {
                            gm[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[p], hv[p], gm[p], 0, 0, 0);
                            gm[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[p], lv[p], gm[p], 0, 0, 0);
                            gm[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lv[p], hv[p], gm[p], 0, 0, 0);
                        }
                    }
                }
            } else if constexpr (F16G && PPW == 1) {
                // One patch: blocks (0,0), (0,1), (1,1) from the same split
                // (see the two-patch case below), three products each.
#pragma unroll
                for (int c = 0; c < MCH; c += 8) {
                    half8 hv[2], lv[2];
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int e = 0; e < 8; e += 2) {
                            const float2v xp = {vm[p][c + e], vm[p][c + e + 1]};
                            const half2v hp = __builtin_convertvector(xp, half2v);
                            const half2v lp = __builtin_convertvector(xp - __builtin_convertvector(hp, float2v), half2v);
                            hv[p][e] = hp[0]; hv[p][e + 1] = hp[1];
                            lv[p][e] = lp[0]; lv[p][e + 1] = lp[1];
                        }
                    gm[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[0], hv[0], gm[0], 0, 0, 0);
                    gm[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[0], lv[0], gm[0], 0, 0, 0);
                    gm[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lv[0], hv[0], gm[0], 0, 0, 0);
                    gm[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[0], hv[1], gm[1], 0, 0, 0);
                    gm[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[0], lv[1], gm[1], 0, 0, 0);
                    gm[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lv[0], hv[1], gm[1], 0, 0, 0);
                    gm[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[1], hv[1], gm[2], 0, 0, 0);
                    gm[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv[1], lv[1], gm[2], 0, 0, 0);
                    gm[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lv[1], hv[1], gm[2], 0, 0, 0);
                }
            } else if constexpr (F16G) {
                // Two patches: each Gram matrix from FP16 matrix-core products
                // of a two-term split, x' = s x = h + l with h = fp16(x')
                // (nearest) and l = fp16(x' - h): G' = H H^T + H L^T + L H^T
                // (the dropped L L^T and the rounding of l are ~2^-22 of
                // |x_i| |x_j|, the size of FP32 accumulation error); G = G' / s^2.
                // s (a power of two, from the plan) keeps |x'| <= 2^14.
                // Lane l supplies k-slots 8 (l / 32) .. + 7 of candidate l % 32
                // from its own half of the coordinates, the same for A and B.
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int c = 0; c < MCH; c += 8) {
                        half8 hv, lv;
#pragma unroll
                        for (int e = 0; e < 8; e += 2) {
                            const float2v xp = {vm[p][c + e], vm[p][c + e + 1]};
                            const half2v hp = __builtin_convertvector(xp, half2v);
                            const half2v lp = split_lo(xp, hp);
                            hv[e] = hp[0]; hv[e + 1] = hp[1];
                            lv[e] = lp[0]; lv[e + 1] = lp[1];
                        }
                        gm[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv, hv, gm[p], 0, 0, 0);
                        gm[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hv, lv, gm[p], 0, 0, 0);
                        gm[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lv, hv, gm[p], 0, 0, 0);
                    }
            } else {
#pragma unroll
                for (int j = 0; j < MCH; ++j) {
                    if constexpr (PPW == 2) {
                        gm[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(vm[0][j], vm[0][j], gm[0], 0, 0, 0);
                        gm[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(vm[1][j], vm[1][j], gm[1], 0, 0, 0);
                    } else {
                        gm[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(vm[0][j], vm[0][j], gm[0], 0, 0, 0);
                        gm[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(vm[0][j], vm[1][j], gm[1], 0, 0, 0);
                        gm[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(vm[1][j], vm[1][j], gm[2], 0, 0, 0);
                    }
                }
            }
            // keep the chunks apart: at most one chunk in flight beyond this one
            if constexpr (MCH < LH) __builtin_amdgcn_sched_barrier(0);
        }
        T hf[2], ef[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            T lo, hi;
            swap_pair<32>(PS ? hs[p] + hs2[p] : hs[p], lo, hi);
            hf[p] = lo + hi;
            if constexpr (!PS) {
                swap_pair<32>(es[p], lo, hi);
                ef[p] = lo + hi;
            }
        }
        // a lane's own candidate is in slot lane / 32 (patch or block).  The
        // iterations run on the split's scaled values: Gram entries and
        // squared norms times s^2, correlations times s t (s = the plan's
        // split scale, t = the measurement's; both powers of two, 1 without
        // the split), so no comparison changes; the coefficients come out
        // times t / s and are scaled back once.
        h[0] = hh ? hf[1] : hf[0];
        if constexpr (!PS) ee[0] = hh ? ef[1] : ef[0];
        // keep the Gram entries in ordinary VGPRs, where a row can be picked
        // by a wavefront-uniform register index
#pragma unroll
        for (int p = 0; p < NGM; ++p)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                float t = gm[p][r];
                asm volatile("" : "+v"(t));
                gm[p][r] = t;
            }
        if constexpr (PS) {
            // squared norms: the Gram diagonal.  Entry (c, c) of a block lives
            // in lane c + 32 ((c / 4) % 2), register 4 (c / 8) + c % 4; the
            // lanes that hold one write their column to LDS, every lane reads
            // its candidate's entry back (one block at a time).
            float *dump = reinterpret_cast<float *>(lds64[wv]);
            const int cc = lane & 31;
            const bool holds = ((cc >> 2) & 1) == hh;
            float dg = 0.f;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int bq = PPW == 2 ? q : 2 * q;
                if (holds) {
#pragma unroll
                    for (int r = 0; r < 16; r += 4)
                        *reinterpret_cast<float4 *>(dump + cc * 16 + r) =
                            make_float4(gm[bq][r], gm[bq][r + 1], gm[bq][r + 2], gm[bq][r + 3]);
                }
                wave_sync();
                const float dv = dump[cc * 16 + 4 * (cc >> 3) + (cc & 3)];
                dg = hh == q ? dv : dg;
                wave_sync();
            }
            ee[0] = dg;
        }
        if constexpr (G01T) {
            // block (0,1) column-major: lane (c, half) writes its rows of
            // column c, four contiguous rows per 16-byte store
            float *gt = &g01_lds[wv][(lane & 31) * G01S + 4 * hh];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<float4 *>(gt + 8 * q) =
                    make_float4(gm[1][4 * q], gm[1][4 * q + 1], gm[1][4 * q + 2], gm[1][4 * q + 3]);
            wave_sync();
        }
    } else if constexpr (!GRAM) {
#pragma unroll
        for (int j = 0; j < LP; ++j) {
            const T sw = w.sqw[j], yh = w.yhat[j];
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                const T xv = v[s][j] * sw;
                const T x = live[s] ? xv : T(0);
                v[s][j] = x;
                h[s] += x * yh;
                ee[s] += x * x;
            }
        }
    } else if (a.hpre) {
        // correlations with y from the batched first-scale GEMM, squared
        // norms from the plan (shared operator: no weights)
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int at = live[s] ? atom[s] : 0;
            const T hv = ((const T *)a.hpre)[bb * (int64_t)a.t + at];
            const T ev = ((const T *)a.nu2)[(int64_t)ph * a.t + at];   // the patch's operator's norms
            h[s] = live[s] ? hv : T(0);
            ee[s] = live[s] ? ev : T(0);
        }
    } else if constexpr (sizeof(T) == 4) {
        // 16 bytes of each candidate row per load (rows and the LDS record
        // are 16-byte aligned, lp is a multiple of 4); the sums keep the
        // coordinate order of the scalar loop below
        for (int j = 0; j < lp; j += 4) {
            const float4 sw = *reinterpret_cast<const float4 *>(&w.sqw[j]);
            const float4 yh = *reinterpret_cast<const float4 *>(&w.yhat[j]);
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                const float4 q = *reinterpret_cast<const float4 *>(src[s] + j);
                const float x0 = live[s] ? q.x * sw.x : 0.f, x1 = live[s] ? q.y * sw.y : 0.f;
                const float x2 = live[s] ? q.z * sw.z : 0.f, x3 = live[s] ? q.w * sw.w : 0.f;
                h[s] += x0 * yh.x;
                h[s] += x1 * yh.y;
                h[s] += x2 * yh.z;
                h[s] += x3 * yh.w;
                ee[s] += x0 * x0;
                ee[s] += x1 * x1;
                ee[s] += x2 * x2;
                ee[s] += x3 * x3;
            }
        }
    } else {
        for (int j = 0; j < lp; ++j) {
            const T sw = w.sqw[j], yh = w.yhat[j];
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                const T xv = src[s][j] * sw;
                const T x = live[s] ? xv : T(0);
                h[s] += x * yh;
                ee[s] += x * x;
            }
        }
    }
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        c[s] = h[s];
        e[s] = ee[s];
        e0[s] = ee[s];
        // inverse norm (FP32: the hardware reciprocal square root, 1 ulp)
        if constexpr (sizeof(T) == 4) nu[s] = __builtin_amdgcn_rsqf(ee[s]);
        else nu[s] = T(1) / sqrt(ee[s]);
        if (!(ee[s] > T(0))) live[s] = false;  // an effective column of zero is never picked
    }

    // The refinement reads the support's vectors RU coordinates per lane at
    // a time.  When one such batch covers every coordinate (KEEP), the values
    // are kept in LDS (lane-major) for x-hat.
    constexpr int RU0 = GRAM ? 4 : ((LP + G - 1) / G > 4 ? 4 : (LP + G - 1) / G);
    constexpr int RU = RU0 * KM > 16 ? (16 / KM > 0 ? 16 / KM : 1) : RU0;
    static_assert(RU >= 1, "refinement batch");
    constexpr bool KEEP = sizeof(T) == 4 && !GRAM && G * RU >= LP;
    __shared__ T keep_lds[KEEP ? W : 1][KEEP ? RU * KM : 1][64];

    // split scale of the matrix-core Gram (1 otherwise): pivots computed
    // from the stored vectors in FP64 are multiplied by it
    const T gs = F16G ? (T)a.gsplit : T(1);

    // ---- OMP iterations (Algorithm 1), unrolled so u and x stay in VGPRs
    T x[KM];          // column gl of L^{-1}
#pragma unroll
    for (int m = 0; m < KM; ++m) x[m] = T(0);
    // alpha_gl = sum_i (L^{-1})_{i,gl} z_i with z = L^{-1} A_Omega^T y, and the
    // squared norm of column gl of L^{-1}, accumulated as the rows appear
    T al = 0, col2 = 0;
    bool active = K > 0;
    int nsel = 0;
    T trg = 0;        // trace of the support's Gram matrix
    // largest and smallest squared pivot (diagonal of L) accepted so far
    T p2max = T(0), p2min = sizeof(T) == 4 ? T(3.0e38f) : T(1.0e300);
    // reduced-precision correlations with y (first scale): slots whose
    // correlation has been re-scored in FP32
    const bool rescore = GRAM && sizeof(T) == 4 && a.hre > 0 && a.hpre != nullptr;
    unsigned exm = 0u;
#pragma unroll
    for (int n = 0; n < KM; ++n) {
        if (n >= kwave) break;
        bool act = active && n < K;
        // proxy: |<a_i, r>| / ||a_i||, lowest atom index on ties
        T best = T(-1);
        int bidx = INT_MAX;
        bool selected = false;
        unsigned long long own = 0;   // lanes that own their group's pick (matrix-core Gram)
        if constexpr (MG) {
            // One candidate per lane: the largest score's bit pattern over the
            // group; the lane that holds it is the pick.  Only when several
            // lanes of a group hold exactly that score (an exact tie) is the
            // lowest atom index among them searched.
            const T sc0 = (act && live[0]) ? fabs(c[0]) * nu[0] : T(-1);
            const int sb = __float_as_int(sc0);
            const int mb = group_max<G>(sb);
            best = __int_as_float(mb);
            const bool tie = (sb == mb) & (mb >= 0);
            own = __ballot(tie);
            bool multi = false;
#pragma unroll
            for (int g = 0; g < PPW; ++g)
                multi = multi || __popcll(G == 64 ? own : ((own >> (g * G)) & 0xFFFFFFFFull)) > 1;
            selected = tie;
            if (multi) {
                const int mi = group_min<G>(tie ? atom[0] : INT_MAX);
                selected = tie && atom[0] == mi;
                own = __ballot(selected);
            }
            act = act && best >= T(0);      // candidates exhausted otherwise
            if (selected) {
#pragma unroll
                for (int m = 0; m < KM; ++m)
                    if (m < n) w.uk[m] = u[0][m];   // entries past n are zero and never read
                w.sc[0] = c[0];
                w.sc[1] = e[0];
                w.sc[2] = e0[0];
            }
        } else {
            if constexpr (GRAM && sizeof(T) == 4) {
                if (rescore) {
                    // The a.hre candidates with the best current scores are
                    // selected, and those whose correlation is still the
                    // reduced-precision one are re-scored in FP32, all lanes
                    // at once (<a_i, y> from the stored vector; a re-scored
                    // slot stays exact).  The pick is the best exactly scored
                    // candidate: the selected ones and any re-scored before.
                    // Selection key: the score with its 11 lowest mantissa
                    // bits dropped, over the inverted atom index (a larger key
                    // is a better score, or an equal one at a lower index);
                    // the a.hre-th largest key of the group is found bit by
                    // bit from the top with ballot counts.
                    unsigned key[NC];
#pragma unroll
                    for (int s = 0; s < NC; ++s) {
                        const T sc = fabs(c[s]) * nu[s];
                        key[s] = (act && live[s] && sc >= T(0))
                                     ? ((((__float_as_uint(sc) >> 11) + 1u) << 12) | (4095u - (unsigned)atom[s]))
                                     : 0u;
                    }
                    unsigned thr = 0u;
                    for (int bit = 31; bit >= 0; --bit) {
                        const unsigned cand = thr | (1u << bit);
                        int cnt = 0;
#pragma unroll
                        for (int s = 0; s < NC; ++s) cnt += group_count<G>(key[s] >= cand, lane);
                        thr = cnt >= a.hre ? cand : thr;
                    }
                    unsigned todo = 0u;
#pragma unroll
                    for (int s = 0; s < NC; ++s)
                        if (key[s] != 0u && key[s] >= thr && !((exm >> s) & 1u)) todo |= 1u << s;
                    if (__ballot(todo != 0u)) {
                        static_assert(G == 64, "Gram-table kernels hold one patch per wavefront");
                        // The wavefront re-scores the selected candidates
                        // together, one at a time: lane l takes coordinates
                        // l, l + 64, ... (the shared dense operator has unit
                        // weights), and the sum goes to every lane.
                        constexpr int NR = LP_GRAM / 64;
                        T yl[NR];
#pragma unroll
                        for (int r = 0; r < NR; ++r) {
                            const int j = lane + 64 * r;
                            yl[r] = j < lp ? w.yhat[j] : T(0);
                        }
#pragma unroll
                        for (int s = 0; s < NC; ++s) {
                            unsigned long long ms = __ballot((todo >> s) & 1u);
                            while (ms) {
                                const int ln = __builtin_ctzll(ms);
                                ms &= ms - 1ull;
                                const int at = __builtin_amdgcn_readlane(atom[s], ln);
                                const T *row = vph + (int64_t)at * lp;
                                T part = T(0);
#pragma unroll
                                for (int r = 0; r < NR; ++r) {
                                    const int j = lane + 64 * r;
                                    if (j < lp) part += row[j] * yl[r];
                                }
                                const T hx = group_sum<64>(part);
                                if (lane == ln) c[s] += hx - ((const T *)a.hpre)[bb * (int64_t)a.t + at];
                            }
                        }
                        exm |= todo;
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                const bool ok = live[s] && (!rescore || ((exm >> s) & 1u));
                const T sc = ok ? fabs(c[s]) * nu[s] : T(-1);
                const bool up = (sc > best) | ((sc == best) & (atom[s] < bidx));
                best = up ? sc : best;
                bidx = up ? atom[s] : bidx;
            }
            best = act ? best : T(-1);
            bidx = act ? bidx : INT_MAX;
            group_argmax<G>(best, bidx);
            act = act && best >= T(0);      // candidates exhausted otherwise
            // the owning lane publishes its vector, its u row and its scalars
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                const bool sel = act && live[s] && atom[s] == bidx;
                selected = selected || sel;
                if (sel) {
                    if constexpr (!GRAM) {
#pragma unroll
                        for (int j = 0; j < LP; ++j) w.vk[j] = v[s][j];
                    }
#pragma unroll
                    for (int m = 0; m < KM; ++m)
                        if (KM > 8 || m < n) w.uk[m] = u[s][m];
                    w.sc[0] = c[s];
                    w.sc[1] = e[s];
                    w.sc[2] = e0[s];
                }
            }
        }
        wave_sync();
        T ck = 0, ek = 0, e0k = 0;
        if (act) { ck = w.sc[0]; ek = w.sc[1]; e0k = w.sc[2]; }
        act = act && n < rank_bound;        // support already spans the space
        T lnn = T(1);
        bool need64 = false;
        if constexpr (sizeof(T) == 4) {
            // the pivot's own condition estimate: ratio of squared diagonals of L
            const T hi = p2max > ek ? p2max : ek;
            const T lo = p2min < ek ? p2min : ek;
            need64 = act && (!(lo > T(0)) || hi > T(1e6) * lo);
        }
        if (act && !need64) {
            if (!(ek > dep_tol<T>() * e0k)) act = false;  // picked atom is dependent
            else lnn = fast_sqrt(ek);
        }
        if constexpr (sizeof(T) == 4) {
            // FP64 pivot: Cholesky of the FP64 Gram of Omega + {k}, one group at a time
            const unsigned long long m64 = __ballot(need64);
            if (m64) {
#pragma unroll
                for (int g = 0; g < PPW; ++g) {
                    if ((m64 >> (g * G)) & 1ull) {
                        GroupLds<T, LPA, KM, PSN> &wg = lds[wv * PPW + g];
                        if (MG ? (selected && gi == g) : (lane == g * G)) wg.sup[n] = MG ? atom[0] : bidx;
                        wave_sync();
                        double *g64 = lds64[wv];
                        double *h64 = g64 + KX * KX;
                        double *pv = h64 + KX;
                        double *gd = pv + KX;
                        const T *vg = (const T *)a.v + (int64_t)__builtin_amdgcn_readlane(ph, g * G) * a.phase_stride;
                        gram64_chol<T>(vg, a.lp, a.l, wg.sqw, wg.yhat, wg.sup, n + 1, lane, g64, h64, pv, gd, false);
                        if (gi == g) {
                            const double piv = pv[n], gkk = gd[n];
                            if (!(piv > 1e-10 * gkk)) act = false;  // dependent in FP64 as well
                            else lnn = (T)sqrt(piv) * gs;
                        }
                        wave_sync();
                    }
                }
            }
        }
        active = active & act;
        // updates run unconditionally; a group that stopped uses inv = 0,
        // which leaves its state unchanged
        const T inv = act ? fast_rcp(lnn) : T(0);
        const T zn = ck * inv;
        const int kb = act ? bidx : INT_MAX;
        // Gram column <a_i, a_k> of every candidate; the selected vector is
        // read in chunks, the next chunk requested before the current one is
        // used, so that few registers hold it at a time
        T gcol[NC];
#pragma unroll
        for (int s = 0; s < NC; ++s) gcol[s] = T(0);
        if constexpr (MG && PPW == 2) {
            // the selected candidate's slot in each patch, then its row of the
            // Gram matrix (symmetric): row k, column gl lives in lane
            // gl + 32 ((k / 4) % 2), register 4 (k / 8) + k % 4
            const unsigned o0 = (unsigned)own, o1 = (unsigned)(own >> 32);
            const int k0 = o0 ? __builtin_ctz(o0) : 0;
            const int k1 = o1 ? __builtin_ctz(o1) : 0;
            const float x0 = gm[0][4 * (k0 >> 3) + (k0 & 3)];
            const float x1 = gm[1][4 * (k1 >> 3) + (k1 & 3)];
            float lo0, hi0, lo1, hi1;
            swap_pair<32>(x0, lo0, hi0);
            swap_pair<32>(x1, lo1, hi1);
            const float g0 = ((k0 >> 2) & 1) ? hi0 : lo0;
            const float g1 = ((k1 >> 2) & 1) ? hi1 : lo1;
            gcol[0] = gi ? g1 : g0;
        } else if constexpr (MG) {
            // one patch: the selected candidate k = 32 bk + kr; lane l needs
            // entry (kr, l % 32) of block (bk, l / 32).  Row kr lives in lane
            // half (kr / 4) % 2, register 4 (kr / 8) + kr % 4; a lane whose
            // own half holds it reads it, the other lane of the pair gets it
            // from its partner, which reads block (bk, 1 - partner half).
            // Block (1,0) is not kept: its row kr is column kr of block
            // (0,1), read from LDS.
            const int k = own ? __builtin_ctzll(own) : 0;
            const int bk = k >> 5, kr = k & 31;
            const int rk = 4 * (kr >> 3) + (kr & 3);
            const int hk = (kr >> 2) & 1;
            // block index by select: only the register index rk is dynamic
            const float b00 = gm[0][rk], b01 = gm[1][rk], b11 = gm[2][rk];
            const float b1 = bk ? b11 : b01;
            const float xo = hh ? b1 : b00;
            const float xt = hh ? b00 : b1;
            float lo, hi;
            swap_pair<32>(xt, lo, hi);
            gcol[0] = hk == hh ? xo : (hh ? lo : hi);
            if (bk) {
                const float t = g01_lds[wv][kr * G01S + (lane & 31)];
                if (!hh) gcol[0] = t;
            }
        } else if constexpr (!GRAM) {
            constexpr int CH = LP <= 16 ? LP : 8;
            T cur[CH], nxt[CH];
            const T *vkp = w.vk;
#pragma unroll
            for (int j = 0; j < CH; ++j) cur[j] = vkp[j];
#pragma unroll
            for (int j0 = 0; j0 < LP; j0 += CH) {
                if (j0 + CH < LP) {
                    // the address of the next chunk is made to depend on the
                    // sums so far, so the compiler cannot request it earlier
                    asm volatile("" : "+v"(vkp) : "v"(gcol[0]));
#pragma unroll
                    for (int j = 0; j < CH; ++j) nxt[j] = vkp[j0 + CH + j];
                }
#pragma unroll
                for (int s = 0; s < NC; ++s)
#pragma unroll
                    for (int j = 0; j < CH; ++j) gcol[s] += v[s][j0 + j] * cur[j];
#pragma unroll
                for (int j = 0; j < CH; ++j) cur[j] = nxt[j];
            }
        } else {
            // the patch's operator's table (plans with several operators)
            const T *gtab = (const T *)a.gram + (int64_t)ph * a.t * a.t;
#pragma unroll
            for (int s = 0; s < NC; ++s)
                if (act & (atom[s] != INT_MAX)) gcol[s] = gtab[(int64_t)bidx * a.t + atom[s]];
        }
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const T g = gcol[s];
            // u rows are zero past n: with up to 8 atoms (and for the
            // matrix-core kernels, built unrolled) the iterations are unrolled
            // and the sum stops at n; otherwise it runs over all KM entries
            // in four independent chains (no loop bound, short dependence)
            T dp[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int m = 0; m < KM; ++m) {
                if ((KM <= 8 || MG) && m >= n) break;
                dp[m & 3] += w.uk[m] * u[s][m];
            }
            const T dot = (dp[0] + dp[1]) + (dp[2] + dp[3]);
            const T un = (g - dot) * inv;
            u[s][n] = un;
            c[s] -= un * zn;
            e[s] -= un * un;
            live[s] = MG ? (live[s] & !(selected & act)) : (live[s] & (atom[s] != kb));
        }
        // column gl of L^{-1}: new entry of the appended row
        T xp[4] = {T(0), T(0), T(0), T(0)};   // x is zero past n as well
#pragma unroll
        for (int m = 0; m < KM; ++m) {
            if ((KM <= 8 || MG) && m >= n) break;
            xp[m & 3] += w.uk[m] * x[m];
        }
        const T xd = (gl == n ? T(1) : T(0)) - ((xp[0] + xp[1]) + (xp[2] + xp[3]));
        x[n] = xd * inv;
        al += x[n] * zn;
        col2 += x[n] * x[n];
        if (MG ? (act & selected) : (act & (gl == 0))) w.sup[n] = MG ? atom[0] : bidx;
        trg += act ? e0k : T(0);
        const T l2 = lnn * lnn;
        p2max = act ? (l2 > p2max ? l2 : p2max) : p2max;
        p2min = act ? (l2 < p2min ? l2 : p2min) : p2min;
        nsel = act ? n + 1 : nsel;
        // one patch per wavefront: iterations are strictly sequential, and
        // keeping the scheduler within one bounds the registers in use
        if constexpr (MG && PPW == 1) __builtin_amdgcn_sched_barrier(0);
    }
    wave_sync();

    // ---- outputs ---------------------------------------------------------
    if (valid && gl == 0) a.kused_out[b] = nsel;
    int *sup_out = a.sup_out + (valid ? b : 0) * (int64_t)a.sup_stride;
    if (!a.last) {
        if (valid)
            for (int i = gl; i < a.sup_count; i += G) sup_out[i] = i < nsel ? w.sup[i] : -1;
        return;
    }
    // coefficients: lane j of the group holds alpha_j (back from the
    // split's scaled units: both factors are powers of two)
    al *= gs / ysc;
    if (gl < nsel) w.alpha[gl] = al;
    // x-hat reuses the refinement's vectors when they are D_high's atoms
    // themselves (finest-scale coordinates that are the signal's samples)
    const bool xkeep = KEEP && a.xhat && a.fold == kFold && a.blk_ident && a.n == a.l;
    bool kept = false;   // the refinement left the support's vectors in LDS
    if constexpr (sizeof(T) == 4) {
        // Condition estimate of the support's Gram matrix G:
        // tr(G) tr(G^{-1}) / n lies between kappa(G) / n and n kappa(G).
        const T trinv = group_sum<G>(col2);
        const double est = nsel > 1 ? (double)trg * (double)trinv / nsel : 1.0;
        // One step of mixed-precision refinement where the FP32 solution can
        // miss the coefficient tolerance.  The FP32 normal equations leave an
        // error of about kappa(G) 2^-24; the residual of the normal
        // equations, r = A_Omega^T (y-hat - A_Omega alpha), is formed in FP64
        // from the stored vectors, and the correction G^{-1} r = L^{-T} L^{-1} r
        // goes through the FP32 factor (lane j holds column j of L^{-1}),
        // which leaves an error of about (kappa(G) 2^-24)^2.
        const bool refine = est > kRefineEst;
        wave_sync();
        if (__ballot(refine)) {
            kept = true;
            double part[KM];
            T alv[KM];
            int sid[KM];
#pragma unroll
            for (int i = 0; i < KM; ++i) {
                const bool in = i < nsel;
                part[i] = 0.0;
                sid[i] = in ? w.sup[i] : 0;
                alv[i] = in ? w.alpha[i] : T(0);
            }
            const T *vv = vph;
            // RU coordinates per lane at a time: all their loads are in
            // flight together (one memory round trip per RU G coordinates)
            for (int t0 = gl; t0 < a.l; t0 += G * RU) {
                T raw[RU][KM];
                // unconditional loads from valid addresses (atoms past nsel
                // read atom 0 and carry alpha 0; coordinates past l are skipped
                // below): a conditional load would become a branch and a wait
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const int t = t0 + u * G;
                    const int tc = t < a.l ? t : 0;
#pragma unroll
                    for (int i = 0; i < KM; ++i) raw[u][i] = vv[(unsigned)(sid[i] * a.lp + tc)];   // t lp < 2^31
                }
                if constexpr (KEEP) {   // a single batch (G RU >= LP >= l)
                    if (xkeep) {
#pragma unroll
                        for (int u = 0; u < RU; ++u)
#pragma unroll
                            for (int i = 0; i < KM; ++i) keep_lds[wv][u * KM + i][lane] = raw[u][i];
                    }
                }
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const int t = t0 + u * G;
                    if (t < a.l) {
                        const double sq = (double)w.sqw[t];
                        double res = (double)w.yhat[t];
#pragma unroll
                        for (int i = 0; i < KM; ++i) res -= (double)alv[i] * ((double)raw[u][i] * sq);
#pragma unroll
                        for (int i = 0; i < KM; ++i) part[i] += ((double)raw[u][i] * sq) * res;
                    }
                }
            }
            T rme = 0;
            if constexpr (G >= 32 && KM >= 8) {
                rme = sums_to_lanes<G, KM>(part, lane);
            } else {
#pragma unroll
                for (int i = 0; i < KM; ++i) {
                    const double ri = group_sum<G>(part[i]);
                    rme = gl == i ? (T)ri : rme;
                }
            }
            T dl = 0;
#pragma unroll
            for (int m = 0; m < KM; ++m) {
                const T wm = group_sum<G>(x[m] * rme);
                dl += x[m] * wm;
            }
            al += dl * (gs * gs);   // x holds L^{-1} of the scaled Gram
        }
        if (gl < nsel) w.alpha[gl] = al;
        // FP64 back-substitution when even the refined FP32 solution would miss
        // the coefficient tolerance (1e-5 relative)
        const bool ill = est > kBackSubEst;
        const unsigned long long mi = __ballot(ill);
        wave_sync();
        if (mi) {
#pragma unroll
            for (int g = 0; g < PPW; ++g) {
                if ((mi >> (g * G)) & 1ull) {
                    GroupLds<T, LPA, KM, PSN> &wg = lds[wv * PPW + g];
                    const int ng = __builtin_amdgcn_readlane(nsel, g * G);
                    double *g64 = lds64[wv];
                    double *h64 = g64 + KX * KX;
                    double *pv = h64 + KX;
                    double *gd = pv + KX;
                    const T *vg = (const T *)a.v + (int64_t)__builtin_amdgcn_readlane(ph, g * G) * a.phase_stride;
                    gram64_chol<T>(vg, a.lp, a.l, wg.sqw, wg.yhat, wg.sup, ng, lane, g64, h64, pv, gd, true);
                    if (lane == g * G)
                        for (int i = 0; i < ng; ++i) wg.alpha[i] = (T)h64[i];
                    wave_sync();
                }
            }
        }
    }
    wave_sync();
    if (!valid) return;
    T *coef = (T *)a.coef_out + b * (int64_t)a.sup_stride;
    for (int i = gl; i < a.sup_count; i += G) {
        sup_out[i] = i < nsel ? w.sup[i] : -1;
        coef[i] = i < nsel ? w.alpha[i] : T(0);
    }
    if (a.xhat) {
        const T *dh = (const T *)a.d_high;
        T *xh = (T *)a.xhat + b * (int64_t)a.n;
        int si[KM];
        T alx[KM];
#pragma unroll
        for (int i = 0; i < KM; ++i) {
            const bool in = i < nsel;
            si[i] = in ? w.sup[i] : 0;
            alx[i] = in ? w.alpha[i] : T(0);
        }
        if constexpr (KEEP) {
            if (xkeep && kept) {
                // the lanes past l wrote nothing and store nothing
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const int j = gl + u * G;
                    T acc = 0;
#pragma unroll
                    for (int i = 0; i < KM; ++i) acc += alx[i] * keep_lds[wv][u * KM + i][lane];
                    if (j < a.n) xh[j] = acc;
                }
                return;
            }
        }
        // XU samples per lane at a time, every selected atom's sample of each
        // requested before any is used (one memory round trip per XU G samples)
        constexpr int XU = (32 / KM < 1 ? 1 : 32 / KM) / (sizeof(T) == 8 ? 2 : 1) > 0
                               ? (32 / KM < 1 ? 1 : 32 / KM) / (sizeof(T) == 8 ? 2 : 1) : 1;
        for (int j0 = gl; j0 < a.n; j0 += G * XU) {
            T d[XU][KM];
#pragma unroll
            for (int u = 0; u < XU; ++u) {
                const int j = j0 + u * G;
                const int jc = j < a.n ? j : 0;   // a valid address; not stored
#pragma unroll
                for (int i = 0; i < KM; ++i) d[u][i] = dh[(unsigned)(si[i] * a.n + jc)];   // T n < 2^31
            }
#pragma unroll
            for (int u = 0; u < XU; ++u) {
                const int j = j0 + u * G;
                T acc = 0;
#pragma unroll
                for (int i = 0; i < KM; ++i) acc += alx[i] * d[u][i];
                if (j < a.n) xh[j] = acc;
            }
        }
    }
}

// Dynamic LDS of one workgroup: per group the patch's observed samples and
// their indicators (2 n values), per wavefront the block table (l + 1 + n).
inline size_t fold_lds_bytes(const ScaleArgs &a, size_t elem, int ppw, int w)
{
    if (a.fold != kFold || a.blk_ident) return 0;
    return elem * (size_t)(w * ppw * 2 * a.n) + sizeof(int) * (size_t)(w * (a.l + 1 + a.n));
}

template <typename T, int LP, int NC, int PPW, int KM, bool GRAM, bool MG = false, bool PS = false>
cspd_status launch_one(const ScaleArgs &a, hipStream_t st)
{
    constexpr int W = waves_per_block<MG>();
    const int64_t waves = (a.b + PPW - 1) / PPW;
    const unsigned grid = (unsigned)((waves + W - 1) / W);
    char label[112];
    const char *mode = GRAM ? "gram" : (MG ? "mfma" : "vec");
    const char *ps = PS ? ",ps" : "";   // candidates split at plan time
    if (a.first && a.last)
        snprintf(label, sizeof(label), "omp_scale<%s,%s,lp%d,nc%d,ppw%d,k%d%s>:full", sizeof(T) == 8 ? "f64" : "f32",
                 mode, GRAM ? a.lp : LP, NC, PPW, KM, ps);
    else
        snprintf(label, sizeof(label), "omp_scale<%s,%s,lp%d,nc%d,ppw%d,k%d%s>:s%d", sizeof(T) == 8 ? "f64" : "f32",
                 mode, GRAM ? a.lp : LP, NC, PPW, KM, ps, a.scale);
    launch_timed(label, k_omp_scale<T, LP, NC, PPW, KM, GRAM, MG, PS>, dim3(grid), dim3(64 * W),
                 (uint32_t)fold_lds_bytes(a, sizeof(T), PPW, W), st, a);
    CSPD_HIP_CHECK(hipGetLastError());
    return CSPD_OK;
}

// Matrix-core Gram kernel: on the plan's pre-split candidates when the scale
// has them (weights 0 or 1: shared dense operator, or single-sample blocks),
// else splitting the weighted candidates in the kernel.
template <int LP, int PPW, int KM>
cspd_status launch_mg(const ScaleArgs &a, hipStream_t st)
{
    if (a.vsplit) return launch_one<float, LP, 1, PPW, KM, false, true, true>(a, st);
    return launch_one<float, LP, 1, PPW, KM, false, true, false>(a, st);
}

}  // namespace scale_impl
}  // namespace cspd
