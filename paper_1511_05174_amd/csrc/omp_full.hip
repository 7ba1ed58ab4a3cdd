// Full-dictionary OMP (Algorithm 1 over every atom of D_high) for
// dictionaries too large for the per-patch register kernels.
//
// A workgroup of four wavefronts owns 32 patches.  Each iteration:
//  1. proxy: C = A^T R for all T atoms and the 32 residuals on FP32 matrix
//     cores (v_mfma_f32_32x32x2f32, one 32-atom tile per step, the tiles
//     dealt round-robin to the four wavefronts); under a per-patch mask the
//     masked column norms are formed the same way, (A o A)^T M, since
//     T x 32 of them do not fit in LDS.  Scores |c| / ||a|| are fused on the
//     accumulators and reduced to a per-patch argmax (lowest index on ties,
//     atoms already in the support excluded through an LDS bit mask);
//  2. support merge, projection and residue: eight threads per patch form
//     the Gram column of the new atom against the support and <a_k, y>,
//     append a row to the Cholesky factor, solve for the coefficients and
//     recompute the residual r = y - A_Omega alpha in the patch's LDS row.
// The MFMA operands use a coordinate permutation shared by both sides: lane
// half h of an operand supplies coordinate h*LP/2 + s at step s, so every lane
// reads a contiguous half row of A and of the residual.
//
// Reduced-precision proxy (a precision option, not in the paper): the proxy
// tiles run on bf16 or fp16 matrix cores (v_mfma_f32_32x32x16_*, FP32
// accumulation) from the plan's 16-bit copy of A and a 16-bit copy of the
// residual (scaled per patch to a maximum of 1, which leaves the argmax
// unchanged and keeps fp16 clear of underflow).  The patch's m best
// reduced-precision candidates (m = rescore_m; an exact top-m under the key
// below) are re-scored with FP32 correlations and norms, and the argmax is
// taken over the re-scored values.  A candidate's key is one 32-bit word:
// its score with the 11 lowest mantissa bits dropped (12 remain, finer than
// the 16-bit products' own error) above its inverted atom index, so a larger
// key is a better score, or an equal one at a lower index.  Each of the eight
// lanes that serve a patch keeps its MM >= m largest keys sorted (insertion is
// a max / min chain, run only for keys above the lane's smallest); the eight
// lists go to LDS, where an entry's rank in the union is its position in its
// own list plus the entries of the other lists above it, and the entries of
// rank below m are the top m.  The eight threads of the patch then re-score
// those m together, one dot product at a time.  Everything after the pick
// stays FP32.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>

#include "cspd_internal.h"

namespace cspd {
namespace full_impl {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

enum { CM_NATIVE = 0, CM_BF16 = 1, CM_F16 = 2 };

constexpr int P = 32;          // patches per workgroup
constexpr int NW = 4;          // wavefronts per workgroup
constexpr int TPP = 8;         // threads per patch in the update phase
constexpr int KX = kMaxK;
constexpr int SELW = 128;      // selection bit-mask words per patch (T <= 4096)

struct FullArgs {
    int64_t b;
    const float *y;            // b x y_stride
    int y_stride;
    const uint8_t *mask;       // b x n or null
    int n;
    const float *v;            // t x lp
    const float *inv_nu;       // t (null under a mask)
    int t;
    int l;
    int lp;
    int rank;                  // rank bound of the measurement space (dense: M)
    const int *kvec;
    int kuni;
    int kcap;                  // = k_max: row stride and cap of k
    int *support;
    float *coef;
    int *k_used;
    float *xhat;
    const float *d_high;       // T x n
    const uint16_t *v_lo;      // t x lp, bf16 or fp16 copy of v (reduced-precision proxy)
    int rescore_m;             // candidates re-scored in FP32 per patch (1..16)
};

__device__ __forceinline__ void sync() { __syncthreads(); }

// sum over the 8 consecutive lanes of a patch (DPP within a half row)
__device__ __forceinline__ float sum8(float v)
{
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
    return v;
}

__device__ __forceinline__ bool beats(float s1, int i1, float s0, int i0)
{
    return (s1 > s0) | ((s1 == s0) & (i1 < i0));
}

// Eight 16-bit values from eight floats (round to nearest even).
template <int CM>
__device__ __forceinline__ void pack8(const float *f, unsigned (&w)[4])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        unsigned lo, hi;
        if constexpr (CM == CM_BF16) {
            unsigned u0 = __float_as_uint(f[2 * i]), u1 = __float_as_uint(f[2 * i + 1]);
            u0 += 0x7fffu + ((u0 >> 16) & 1u);
            u1 += 0x7fffu + ((u1 >> 16) & 1u);
            lo = u0 >> 16;
            hi = u1 >> 16;
        } else {
            const _Float16 h0 = (_Float16)f[2 * i], h1 = (_Float16)f[2 * i + 1];
            lo = *reinterpret_cast<const unsigned short *>(&h0);
            hi = *reinterpret_cast<const unsigned short *>(&h1);
        }
        w[i] = lo | (hi << 16);
    }
}

template <int CM>
__device__ __forceinline__ f32x16 mfma16(const unsigned (&x)[4], const unsigned (&y)[4], f32x16 acc)
{
    if constexpr (CM == CM_BF16) {
        bf16x8 xa, ya;
        __builtin_memcpy(&xa, x, 16);
        __builtin_memcpy(&ya, y, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, ya, acc, 0, 0, 0);
    } else {
        f16x8 xa, ya;
        __builtin_memcpy(&xa, x, 16);
        __builtin_memcpy(&ya, y, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(xa, ya, acc, 0, 0, 0);
    }
}

// Best (score, atom) over the eight consecutive lanes of a patch.
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(float &s, int &i)
{
    const float os = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s), CTRL, 0xF, 0xF, false));
    const int oi = __builtin_amdgcn_mov_dpp(i, CTRL, 0xF, 0xF, false);
    const bool take = beats(os, oi, s, i);
    s = take ? os : s;
    i = take ? oi : i;
}

__device__ __forceinline__ void argmax8(float &s, int &i)
{
    argmax_dpp<0xB1>(s, i);
    argmax_dpp<0x4E>(s, i);
    argmax_dpp<0x141>(s, i);
}

template <int LP, int KM, bool MASK, int CM, int MM>
__global__ __launch_bounds__(64 * NW) void k_omp_full(FullArgs a)
{
    constexpr int HL = LP / 2;            // coordinates per operand half
    constexpr int RS = LP + 4;            // LDS row stride
    constexpr int CP = LP / TPP;          // coordinates per update thread
    constexpr int NL = KM * (KM + 1) / 2;
    __shared__ float s_r[P][RS];
    __shared__ float s_y[P][RS];
    __shared__ float s_m[MASK ? P : 1][MASK ? RS : 1];
    __shared__ unsigned s_sel[P][SELW];
    __shared__ float s_bs[NW][P];
    __shared__ int s_bi[NW][P];
    __shared__ int s_k[P];
    __shared__ float s_l[P][NL];
    __shared__ float s_z[P][KM];
    __shared__ float s_al[P][KM];
    __shared__ int s_sup[P][KM];
    __shared__ int s_n[P], s_kk[P], s_live[P];
    // reduced-precision pools: 8 sorted lists of MM (score, atom) per patch,
    // and the patch's top m in rank order (-1: fewer valid candidates)
    constexpr bool RP = CM != CM_NATIVE;
    __shared__ unsigned s_pk[RP ? P : 1][RP ? NW * 2 : 1][RP ? MM : 1];
    __shared__ int s_top[RP ? P : 1][RP ? MM : 1];
    const int mtop = RP ? (a.rescore_m < MM ? (a.rescore_m > 0 ? a.rescore_m : 1) : MM) : 1;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * P;
    const int ntiles = (a.t + 31) / 32;

    // ---- patch set-up ------------------------------------------------------
    for (int i = tid; i < P * SELW; i += 64 * NW) s_sel[i / SELW][i % SELW] = 0u;
    for (int i = tid; i < P * LP; i += 64 * NW) {
        const int p = i / LP, j = i % LP;
        const int64_t b = b0 + p;
        float yv = 0.f, mv = 1.f;
        if (b < a.b && j < a.l) {
            yv = a.y[b * (int64_t)a.y_stride + j];
            if constexpr (MASK) { mv = a.mask[b * (int64_t)a.n + j] ? 1.f : 0.f; yv *= mv; }
        } else {
            mv = 0.f;
        }
        s_y[p][j] = yv;
        s_r[p][j] = yv;
        if constexpr (MASK) s_m[p][j] = mv;
    }
    if (tid < P) {
        const int64_t b = b0 + tid;
        int k = 0;
        if (b < a.b) {
            k = a.kvec ? a.kvec[b] : a.kuni;
            k = k < a.kcap ? k : a.kcap;
            k = k < KM ? k : KM;
            k = k < a.t ? k : a.t;
            k = k > 0 ? k : 0;
        }
        s_kk[tid] = k;
        s_n[tid] = 0;
        s_live[tid] = k > 0;
    }
    sync();
    int kmax = 0;
    for (int p = 0; p < P; ++p) kmax = s_kk[p] > kmax ? s_kk[p] : kmax;
    int rank = a.rank;
    (void)rank;

    const int up = tid / TPP;         // patch of this thread in the update phase
    const int us = tid % TPP;         // its slice of the coordinates
    float mk[CP];
#pragma unroll
    for (int q = 0; q < CP; ++q) mk[q] = MASK ? s_m[up][us * CP + q] : 1.f;
    int rank_p = MASK ? 0 : a.rank;
    if constexpr (MASK) {
        float cnt = 0.f;
#pragma unroll
        for (int q = 0; q < CP; ++q) cnt += mk[q];
        rank_p = (int)sum8(cnt);
    }

    for (int it = 0; it < kmax; ++it) {
        // ---- 1. proxy on matrix cores ----------------------------------------
        const int pp = lane & 31;         // patch column of this lane
        const int h = lane >> 5;          // operand half
        float rb[HL];
        float mb[MASK ? HL : 1];
#pragma unroll
        for (int s = 0; s < HL; ++s) {
            rb[s] = s_r[pp][h * HL + s];
            if constexpr (MASK) mb[s] = s_m[pp][h * HL + s];
        }
        float bs = -1.f;
        int bi = INT_MAX;
        unsigned lk[RP ? MM : 1];   // this lane's largest keys, sorted (0: empty)
#pragma unroll
        for (int q = 0; q < (RP ? MM : 1); ++q) lk[q] = 0u;
        if constexpr (RP) {
            for (int i = tid; i < P * MM; i += 64 * NW) s_top[i / MM][i % MM] = -1;
        }
        const bool plive = s_live[pp] != 0;
        unsigned rlo[CM != CM_NATIVE ? HL / 8 : 1][4];
        if constexpr (CM != CM_NATIVE) {
            // 16-bit residual half of the lane's patch, scaled to max |r| = 1
            float mx = 0.f;
#pragma unroll
            for (int s = 0; s < HL; ++s) mx = fmaxf(mx, fabsf(rb[s]));
            {
                auto rs = __builtin_amdgcn_permlane32_swap(__float_as_int(mx), __float_as_int(mx), false, false);
                mx = fmaxf(__int_as_float(rs[0]), __int_as_float(rs[1]));
            }
            const float sc = mx > 0.f ? 1.f / mx : 0.f;
#pragma unroll
            for (int g = 0; g < HL / 8; ++g) {
                float f[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) f[j] = rb[8 * g + j] * sc;
                pack8<CM>(f, rlo[g]);
            }
        }
        for (int t = wave; t < ntiles; t += NW) {
            const int arow = t * 32 + (lane & 31);
            f32x16 acc = {};
            f32x16 nac = {};
            if constexpr (CM == CM_NATIVE || MASK) {
                const float *src = a.v + (int64_t)(arow < a.t ? arow : 0) * a.lp + h * HL;
                float ab[HL];
#pragma unroll
                for (int s = 0; s < HL; s += 4) {
                    const float4 q = *reinterpret_cast<const float4 *>(src + s);
                    ab[s] = q.x; ab[s + 1] = q.y; ab[s + 2] = q.z; ab[s + 3] = q.w;
                }
#pragma unroll
                for (int s = 0; s < HL; ++s) {
                    if constexpr (CM == CM_NATIVE) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ab[s], rb[s], acc, 0, 0, 0);
                    if constexpr (MASK) nac = __builtin_amdgcn_mfma_f32_32x32x2f32(ab[s] * ab[s], mb[s], nac, 0, 0, 0);
                }
            }
            if constexpr (CM != CM_NATIVE) {
                const uint16_t *srl = a.v_lo + (int64_t)(arow < a.t ? arow : 0) * a.lp + h * HL;
#pragma unroll
                for (int g = 0; g < HL / 8; ++g) {
                    const uint4 q = *reinterpret_cast<const uint4 *>(srl + 8 * g);
                    const unsigned x[4] = {q.x, q.y, q.z, q.w};
                    acc = mfma16<CM>(x, rlo[g], acc);
                }
            }
            const unsigned selw = s_sel[pp][t];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * h + (r & 3);
                const int atom = t * 32 + row;
                float inv;
                if constexpr (MASK) inv = nac[r] > 0.f ? 1.f / sqrtf(nac[r]) : -1.f;
                else inv = atom < a.t ? a.inv_nu[atom] : -1.f;
                float sc = fabsf(acc[r]) * inv;
                const bool ok = plive & (atom < a.t) & (inv > 0.f) & (((selw >> row) & 1u) == 0u);
                sc = ok ? sc : -1.f;
                if constexpr (RP) {
                    // key: score bits >> 11 (plus one, so 0 means none) over
                    // the inverted atom index (atoms < 4096)
                    const unsigned key = sc >= 0.f ? ((((__float_as_uint(sc) >> 11) + 1u) << 12) | (4095u - (unsigned)atom))
                                                   : 0u;
                    if (key > lk[MM - 1]) {
                        unsigned x = key;
#pragma unroll
                        for (int q = 0; q < MM; ++q) {
                            const unsigned hi = x > lk[q] ? x : lk[q];
                            x = x > lk[q] ? lk[q] : x;
                            lk[q] = hi;
                        }
                    }
                } else if (sc > bs) {
                    bs = sc;
                    bi = atom;
                }
            }
        }
        if constexpr (RP) {
            // the eight sorted pools of each patch to LDS
#pragma unroll
            for (int q = 0; q < MM; ++q) s_pk[pp][wave * 2 + h][q] = lk[q];
            sync();
            {
                // rank of each own entry in the union; the top m by rank
                const int upp = tid / TPP, uss = tid % TPP;
                for (int q = 0; q < mtop; ++q) {
                    const unsigned ek = s_pk[upp][uss][q];
                    if (ek == 0u) break;
                    int rank = q;
                    for (int j = 0; j < NW * 2 && rank < mtop; ++j) {
                        if (j == uss) continue;
                        for (int r = 0; r < MM && s_pk[upp][j][r] > ek; ++r) ++rank;
                    }
                    if (rank < mtop) s_top[upp][rank] = 4095 - (int)(ek & 4095u);
                }
            }
            sync();
            {
                // FP32 re-score of the top m by the patch's eight threads
                const int upp = tid / TPP, uss = tid % TPP;
                float best = -1.f;
                int bidx = INT_MAX;
                for (int j = 0; j < mtop; ++j) {
                    const int atom = s_top[upp][j];
                    if (atom < 0) break;
                    const float *ar = a.v + (int64_t)atom * a.lp + uss * CP;
                    float c = 0.f, nn = 0.f;
                    float vv[CP];
                    if constexpr (CP % 4 == 0) {
#pragma unroll
                        for (int q = 0; q < CP; q += 4) {
                            const float4 v4 = *reinterpret_cast<const float4 *>(ar + q);
                            vv[q] = v4.x; vv[q + 1] = v4.y; vv[q + 2] = v4.z; vv[q + 3] = v4.w;
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < CP; ++q) vv[q] = ar[q];
                    }
#pragma unroll
                    for (int q = 0; q < CP; ++q) {
                        c += vv[q] * s_r[upp][uss * CP + q];
                        if constexpr (MASK) nn += vv[q] * vv[q] * mk[q];
                    }
                    c = sum8(c);
                    float inv;
                    if constexpr (MASK) {
                        nn = sum8(nn);
                        inv = nn > 0.f ? 1.f / sqrtf(nn) : -1.f;
                    } else {
                        inv = a.inv_nu[atom];
                    }
                    const float sc = inv > 0.f ? fabsf(c) * inv : -1.f;
                    if (beats(sc, atom, best, bidx)) { best = sc; bidx = atom; }
                }
                if (uss == 0) {
                    const bool go = s_live[upp] && best >= 0.f && s_n[upp] < s_kk[upp];
                    s_k[upp] = go ? bidx : -1;
                }
            }
            sync();
        } else {
        // lanes l and l + 32 hold the same patch
        {
            auto rs = __builtin_amdgcn_permlane32_swap(__float_as_int(bs), __float_as_int(bs), false, false);
            auto ri = __builtin_amdgcn_permlane32_swap(bi, bi, false, false);
            const float s0 = __int_as_float(rs[0]), s1 = __int_as_float(rs[1]);
            const bool t1 = beats(s1, ri[1], s0, ri[0]);
            bs = t1 ? s1 : s0;
            bi = t1 ? ri[1] : ri[0];
        }
        if (lane < 32) { s_bs[wave][lane] = bs; s_bi[wave][lane] = bi; }
        sync();
        if (tid < P) {
            float b = s_bs[0][tid];
            int i = s_bi[0][tid];
            for (int w = 1; w < NW; ++w)
                if (beats(s_bs[w][tid], s_bi[w][tid], b, i)) { b = s_bs[w][tid]; i = s_bi[w][tid]; }
            const bool go = s_live[tid] && b >= 0.f && s_n[tid] < s_kk[tid];
            s_k[tid] = go ? i : -1;
        }
        sync();
        }

        // ---- 2. support merge, projection and residue ------------------------
        const int k = s_k[up];
        const int n = s_n[up];
        if (k >= 0) {
            float ak[CP];
            const float *ka = a.v + (int64_t)k * a.lp + us * CP;
#pragma unroll
            for (int q = 0; q < CP; ++q) ak[q] = ka[q] * mk[q];
            float g[KM];
#pragma unroll
            for (int m = 0; m < KM; ++m) {
                float part = 0.f;
                if (m < n) {
                    const float *am = a.v + (int64_t)s_sup[up][m] * a.lp + us * CP;
#pragma unroll
                    for (int q = 0; q < CP; ++q) part += am[q] * ak[q];
                }
                g[m] = part;
            }
            float pk = 0.f, ph = 0.f;
#pragma unroll
            for (int q = 0; q < CP; ++q) { pk += ak[q] * ak[q]; ph += ak[q] * s_y[up][us * CP + q]; }
#pragma unroll
            for (int m = 0; m < KM; ++m) g[m] = sum8(g[m]);
            const float gkk = sum8(pk);
            const float hk = sum8(ph);
            // w = L^{-1} g, pivot = gkk - |w|^2
            float wv[KM];
            float ww = 0.f;
#pragma unroll
            for (int i = 0; i < KM; ++i) {
                wv[i] = 0.f;
                if (i < n) {
                    float s = g[i];
#pragma unroll
                    for (int j = 0; j < i; ++j) s -= s_l[up][i * (i + 1) / 2 + j] * wv[j];
                    wv[i] = s / s_l[up][i * (i + 1) / 2 + i];
                    ww += wv[i] * wv[i];
                }
            }
            const float piv = gkk - ww;
            const bool dep = !(piv > 1e-5f * gkk) || n >= rank_p;
            if (dep) {
                if (us == 0) s_live[up] = 0;
            } else {
                const float lnn = sqrtf(piv);
                float zw = 0.f;
#pragma unroll
                for (int j = 0; j < KM; ++j) zw += j < n ? wv[j] * s_z[up][j] : 0.f;
                const float zn = (hk - zw) / lnn;
                // coefficients: L^T alpha = z with the new row appended
                float al[KM];
#pragma unroll
                for (int i = KM - 1; i >= 0; --i) {
                    al[i] = 0.f;
                    if (i <= n) {
                        float s = i == n ? zn : s_z[up][i];
#pragma unroll
                        for (int m = i + 1; m < KM; ++m) {
                            if (m <= n) {
                                const float lmi = m == n ? wv[i] : s_l[up][m * (m + 1) / 2 + i];
                                s -= lmi * al[m];
                            }
                        }
                        al[i] = s / (i == n ? lnn : s_l[up][i * (i + 1) / 2 + i]);
                    }
                }
                // residue on this thread's coordinates
                float rr[CP];
#pragma unroll
                for (int q = 0; q < CP; ++q) rr[q] = s_y[up][us * CP + q];
#pragma unroll
                for (int m = 0; m < KM; ++m) {
                    if (m <= n) {
                        const int atom = m == n ? k : s_sup[up][m];
                        const float *am = a.v + (int64_t)atom * a.lp + us * CP;
#pragma unroll
                        for (int q = 0; q < CP; ++q) rr[q] -= al[m] * am[q] * mk[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < CP; ++q) s_r[up][us * CP + q] = rr[q];
                if (us == 0) {
                    for (int j = 0; j < n; ++j) s_l[up][n * (n + 1) / 2 + j] = wv[j];
                    s_l[up][n * (n + 1) / 2 + n] = lnn;
                    s_z[up][n] = zn;
#pragma unroll
                    for (int m = 0; m < KM; ++m)
                        if (m <= n) s_al[up][m] = al[m];
                    s_sup[up][n] = k;
                    s_sel[up][k >> 5] |= 1u << (k & 31);
                    s_n[up] = n + 1;
                }
            }
        }
        sync();
    }

    // ---- outputs ---------------------------------------------------------------
    const int64_t b = b0 + up;
    if (b >= a.b) return;
    const int nsel = s_n[up];
    if (us == 0) a.k_used[b] = nsel;
    for (int i = us; i < a.kcap; i += TPP) {
        a.support[b * (int64_t)a.kcap + i] = i < nsel ? s_sup[up][i] : -1;
        a.coef[b * (int64_t)a.kcap + i] = i < nsel ? s_al[up][i] : 0.f;
    }
    if (a.xhat) {
        for (int j = us; j < a.n; j += TPP) {
            float acc = 0.f;
            for (int i = 0; i < nsel; ++i) acc += s_al[up][i] * a.d_high[(int64_t)s_sup[up][i] * a.n + j];
            a.xhat[b * (int64_t)a.n + j] = acc;
        }
    }
}

template <int LP, int KM, bool MASK, int CM, int MM>
cspd_status launch(const FullArgs &a, hipStream_t st)
{
    const unsigned grid = (unsigned)((a.b + P - 1) / P);
    char label[96];
    const char *ty = CM == CM_BF16 ? "bf16" : (CM == CM_F16 ? "f16" : "f32");
    snprintf(label, sizeof(label), "omp_full_mfma<%s,lp%d,k%d%s,m%d>:full", ty, LP, KM, MASK ? ",mask" : "",
             CM == CM_NATIVE ? 0 : MM);
    launch_timed(label, k_omp_full<LP, KM, MASK, CM, MM>, dim3(grid), dim3(64 * NW), 0u, st, a);
    CSPD_HIP_CHECK(hipGetLastError());
    return CSPD_OK;
}

template <int LP, int KM, int CM, int MM>
cspd_status by_mask(const FullArgs &a, bool mask, hipStream_t st)
{
    return mask ? launch<LP, KM, true, CM, MM>(a, st) : launch<LP, KM, false, CM, MM>(a, st);
}

template <int LP, int KM>
cspd_status by_mode(const FullArgs &a, bool mask, int corr, int rr, hipStream_t st)
{
    if constexpr (LP >= 16) {
        if (corr == CSPD_CORR_BF16_RESCORE)
            return rr <= 8 ? by_mask<LP, KM, CM_BF16, 8>(a, mask, st) : by_mask<LP, KM, CM_BF16, 16>(a, mask, st);
        if (corr == CSPD_CORR_F16_RESCORE)
            return rr <= 8 ? by_mask<LP, KM, CM_F16, 8>(a, mask, st) : by_mask<LP, KM, CM_F16, 16>(a, mask, st);
    }
    return by_mask<LP, KM, CM_NATIVE, 1>(a, mask, st);
}

template <int LP>
cspd_status by_k(const FullArgs &a, int kmax, bool mask, int corr, int rr, hipStream_t st)
{
    if (kmax <= 8) return by_mode<LP, 8>(a, mask, corr, rr, st);
    return by_mode<LP, 16>(a, mask, corr, rr, st);
}

}  // namespace full_impl

bool full_mfma_fits(const cspd_plan_s *p)
{
    const ScalePlan &sc = p->sc[p->s - 1];
    return p->dtype == CSPD_F32 && sc.t <= 32 * full_impl::SELW &&
           (sc.lp == 16 || sc.lp == 32 || sc.lp == 64 || sc.lp == 128);
}

cspd_status launch_full_mfma(const cspd_plan_s *p, int64_t b, const void *y, const uint8_t *mask,
                             const int *kvec, int kuni, int *support, void *coef, int *k_used,
                             void *xhat, hipStream_t stream)
{
    using namespace full_impl;
    if (!full_mfma_fits(p))
        return set_error(CSPD_E_UNSUPPORTED, "full search over %d atoms of length %d is not built for this plan",
                         p->sc[p->s - 1].t, p->sc[p->s - 1].l);
    if (b <= 0) return CSPD_OK;
    const ScalePlan &sc = p->sc[p->s - 1];
    FullArgs a{};
    a.b = b;
    a.y = (const float *)y;
    a.y_stride = p->m;
    a.mask = p->phi_kind == CSPD_PHI_MASK ? mask : nullptr;
    a.n = p->n;
    a.v = (const float *)sc.v;
    a.inv_nu = (const float *)sc.inv_nu;
    a.t = sc.t;
    a.l = sc.l;
    a.lp = sc.lp;
    a.rank = p->phi_kind == CSPD_PHI_DENSE ? p->m : sc.l;
    a.kvec = kvec;
    a.kuni = kuni;
    a.kcap = p->k_max;
    a.support = support;
    a.coef = (float *)coef;
    a.k_used = k_used;
    a.xhat = (float *)xhat;
    a.d_high = (const float *)p->d_high;
    a.v_lo = (const uint16_t *)sc.v_lo;
    const int kmax = kvec ? p->k_max : kuni;
    const bool m = a.mask != nullptr;
    const int corr = sc.v_lo ? p->corr_mode : CSPD_CORR_NATIVE;
    const int rr = p->rescore_m;    // top m re-scored per patch (pool lists of 8 or 16 per lane)
    a.rescore_m = rr;
    switch (sc.lp) {
        case 16: return by_k<16>(a, kmax, m, corr, rr, stream);
        case 32: return by_k<32>(a, kmax, m, corr, rr, stream);
        case 64: return by_k<64>(a, kmax, m, corr, rr, stream);
        case 128: return by_k<128>(a, kmax, m, corr, rr, stream);
        default: return CSPD_E_UNSUPPORTED;
    }
}

}  // namespace cspd
