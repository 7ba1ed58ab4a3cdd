// Dictionary update of K-SVD (Section III-E: the cross-scale dictionaries are
// learned by K-SVD on the down-sampled training set, then by the same update
// with the sparse-approximation step restricted to the children of the
// coarse support).  The sparse-approximation step is the library's OMP; this
// file holds the update that follows it.
//
// One sweep, atoms in index order, each update seeing the previous ones:
//   users of atom k   = the (signal, slot) pairs whose support holds k
//   E_k               = R_users + s_k d_k^T   (the error without atom k)
//   d_k               = leading left singular vector of E_k^T (sign kept
//                       towards the old atom)
//   s_k               = E_k d_k,  R_users = E_k - s_k d_k^T
// The residual R = X - D S is formed once per sweep.  The users are listed
// per atom by a stable radix sort of the support entries (atom key, entry
// index value), so each list is in signal order and the sweep is
// deterministic.  The singular vector is the leading eigenvector of the
// N x N matrix C = E_k^T E_k: its upper triangle is accumulated in FP64 by PG
// workgroups over slices of the users, summed in a fixed order by one
// workgroup, which runs the power iteration (FP64, one wavefront) from the
// old atom until it stops moving; PG workgroups then update the users.  Three
// launches per atom, in order on the stream.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "cspd_internal.h"

namespace cspd {
namespace ksvd_impl {

constexpr int NMAX = 64;    // longest atom (C is NMAX x NMAX doubles in LDS)
constexpr int BS = 256;     // threads of the per-atom kernel
constexpr int UCH = 32;     // users staged in LDS at a time

__global__ void k_residual(const float *__restrict__ x, const float *__restrict__ d, const int *__restrict__ sup,
                           const float *__restrict__ coef, int kstride, int64_t p, int n, float *__restrict__ r)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * n) return;
    const int64_t row = t / n;
    const int i = (int)(t - row * n);
    float acc = x[t];
    for (int j = 0; j < kstride; ++j) {
        const int a = sup[row * kstride + j];
        if (a >= 0) acc -= coef[row * kstride + j] * d[(int64_t)a * n + i];
    }
    r[t] = acc;
}

// keys: atom of each support entry (T for an unused slot); values: entry index
__global__ void k_keys(const int *__restrict__ sup, int64_t entries, int t_atoms, int *__restrict__ key,
                       int *__restrict__ val, int *__restrict__ count)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= entries) return;
    const int a = sup[e];
    const bool ok = a >= 0 && a < t_atoms;
    key[e] = ok ? a : t_atoms;
    val[e] = (int)e;
    if (ok) atomicAdd(&count[a], 1);
}

__global__ void k_fill_zero_i32(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

constexpr int NUT = NMAX * (NMAX + 1) / 2;   // upper-triangle entries of C
constexpr int PG = 32;                         // workgroups that share one atom's Gram accumulation
constexpr int EPT = (NUT + BS - 1) / BS;       // upper-triangle entries per thread

// tab[q] = i | j << 8 for upper-triangle entry q = (i, j), i <= j, of an
// n x n matrix (row-major over the triangle)
__global__ void k_tri_table(int n, int *tab)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int base = i * n - i * (i - 1) / 2;
    for (int j = i; j < n; ++j) tab[base + j - i] = i | (j << 8);
}

// Part g of C = sum over atom k's users of e e^T, e = r + s d_k: the users
// [g per, (g + 1) per), upper triangle, FP64, to part[g][*].
__global__ __launch_bounds__(BS) void k_atom_gram(int k, int n, int kstride, const int *__restrict__ off,
                                                  const int *__restrict__ count, const int *__restrict__ ent,
                                                  const float *__restrict__ d, const float *__restrict__ coef,
                                                  const float *__restrict__ r, const int *__restrict__ tab,
                                                  double *__restrict__ part)
{
    __shared__ float eu[UCH][NMAX];
    __shared__ float dk[NMAX];
    const int tid = threadIdx.x;
    const int m = count[k];
    const int per = (m + PG - 1) / PG;
    const int u_beg = blockIdx.x * per;
    const int u_end = u_beg + per < m ? u_beg + per : m;
    const int nut = n * (n + 1) / 2;
    double acc[EPT];
    int ii[EPT], jj[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        acc[e] = 0.0;
        const int q = tid + e * BS;
        const int ij = q < nut ? tab[q] : 0;
        ii[e] = ij & 255;
        jj[e] = ij >> 8;
    }
    for (int i = tid; i < n; i += BS) dk[i] = d[(int64_t)k * n + i];
    __syncthreads();
    for (int u0 = u_beg; u0 < u_end; u0 += UCH) {
        const int nu = u_end - u0 < UCH ? u_end - u0 : UCH;
        for (int q = tid; q < nu * n; q += BS) {
            const int uu = q / n, i = q - uu * n;
            const int e = ent[off[k] + u0 + uu];
            eu[uu][i] = r[(int64_t)(e / kstride) * n + i] + coef[e] * dk[i];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if (tid + e * BS < nut) {
                double a = acc[e];
                for (int uu = 0; uu < nu; ++uu) a += (double)eu[uu][ii[e]] * (double)eu[uu][jj[e]];
                acc[e] = a;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e)
        if (tid + e * BS < nut) part[(int64_t)blockIdx.x * NUT + tid + e * BS] = acc[e];
}

// One atom (one workgroup): sums the Gram parts, power iteration, the
// users' coefficients and residual, the new atom.
__global__ __launch_bounds__(BS) void k_atom(int k, int n, const int *__restrict__ count, float *__restrict__ d,
                                             float *__restrict__ dold, const double *__restrict__ part,
                                             const int *__restrict__ tab, int max_iter, double tol)
{
    __shared__ double c[NMAX * NMAX];
    __shared__ float dk[NMAX];
    __shared__ double v[NMAX];
    const int tid = threadIdx.x;
    const int m = count[k];
    if (m == 0) return;   // an unused atom keeps its value
    const int nut = n * (n + 1) / 2;
    for (int i = tid; i < n; i += BS) {
        dk[i] = d[(int64_t)k * n + i];
        dold[i] = dk[i];
    }
    // C from the parts, in a fixed order (deterministic)
    for (int q = tid; q < nut; q += BS) {
        double a = 0.0;
        for (int g = 0; g < PG; ++g) a += part[(int64_t)g * NUT + q];
        const int ij = tab[q];
        const int i = ij & 255, j = ij >> 8;
        c[i * n + j] = a;
        c[j * n + i] = a;
    }
    __syncthreads();
    // power iteration from the old atom, v <- C v / ||C v|| until it stops
    // moving, on the first wavefront alone (lane i owns row i; the other
    // wavefronts wait at the barrier below): no workgroup barrier per step
    if (tid < 64) {
        const int i = tid;
        double vi = i < n ? (double)dk[i] : 0.0;
        for (int it = 0; it < max_iter; ++it) {
            if (i < n) v[i] = vi;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // C is stored in full and symmetric: lane i reads column i
            // (c[j n + i]), so the wavefront's reads of one j are consecutive
            // words, not one bank 64 times over
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            if (i < n) {
                int j = 0;
                for (; j + 4 <= n; j += 4) {
                    a0 += c[j * n + i] * v[j];
                    a1 += c[(j + 1) * n + i] * v[j + 1];
                    a2 += c[(j + 2) * n + i] * v[j + 2];
                    a3 += c[(j + 3) * n + i] * v[j + 3];
                }
                for (; j < n; ++j) a0 += c[j * n + i] * v[j];
            }
            const double wi = (a0 + a1) + (a2 + a3);
            double nn = wi * wi;
            for (int o = 32; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 64);
            const double nrm = sqrt(nn);
            const double nv = nrm > 0.0 ? wi / nrm : 0.0;
            double dd = (nv - vi) * (nv - vi);
            for (int o = 32; o > 0; o >>= 1) dd += __shfl_xor(dd, o, 64);
            vi = nv;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (!(nrm > 0.0) || sqrt(dd) < tol) break;
        }
        // sign towards the old atom
        double sp = i < n ? vi * (double)dk[i] : 0.0;
        for (int o = 32; o > 0; o >>= 1) sp += __shfl_xor(sp, o, 64);
        if (i < n) v[i] = sp < 0.0 ? -vi : vi;
    }
    __syncthreads();
    for (int i = tid; i < n; i += BS) d[(int64_t)k * n + i] = (float)v[i];
}

// The users of atom k, in PG slices: e = r + s_old d_old, s = e . d_new,
// r = e - s d_new (the new atom is already in d, the old one in dold).
__global__ __launch_bounds__(BS) void k_atom_users(int k, int n, int kstride, const int *__restrict__ off,
                                                   const int *__restrict__ count, const int *__restrict__ ent,
                                                   const float *__restrict__ d, const float *__restrict__ dold,
                                                   float *__restrict__ coef, float *__restrict__ r)
{
    __shared__ float eu[UCH][NMAX];
    __shared__ float su[UCH];
    __shared__ float dn[NMAX], dp[NMAX];
    const int tid = threadIdx.x;
    const int m = count[k];
    if (m == 0) return;
    const int per = (m + PG - 1) / PG;
    const int u_beg = blockIdx.x * per;
    const int u_end = u_beg + per < m ? u_beg + per : m;
    const int base = off[k];
    for (int i = tid; i < n; i += BS) {
        dn[i] = d[(int64_t)k * n + i];
        dp[i] = dold[i];
    }
    __syncthreads();
    for (int u0 = u_beg; u0 < u_end; u0 += UCH) {
        const int nu = u_end - u0 < UCH ? u_end - u0 : UCH;
        for (int q = tid; q < nu * n; q += BS) {
            const int uu = q / n, i = q - uu * n;
            const int e = ent[base + u0 + uu];
            eu[uu][i] = r[(int64_t)(e / kstride) * n + i] + coef[e] * dp[i];
        }
        __syncthreads();
        if (tid < nu) {
            double acc = 0.0;
            for (int i = 0; i < n; ++i) acc += (double)eu[tid][i] * (double)dn[i];
            su[tid] = (float)acc;
        }
        __syncthreads();
        for (int q = tid; q < nu * n; q += BS) {
            const int uu = q / n, i = q - uu * n;
            const int e = ent[base + u0 + uu];
            r[(int64_t)(e / kstride) * n + i] = eu[uu][i] - su[uu] * dn[i];
        }
        if (tid < nu) coef[ent[base + u0 + tid]] = su[tid];
        __syncthreads();
    }
}

}  // namespace ksvd_impl
}  // namespace cspd

using namespace cspd;
using namespace cspd::ksvd_impl;

extern "C" {

cspd_status cspd_ksvd_update(const float *x, int64_t p, int32_t n, float *dict, int32_t t_atoms,
                             const int32_t *support, float *coef, int32_t kstride, void *hip_stream)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (p < 0 || n < 1 || n > NMAX || t_atoms < 1 || kstride < 1)
            return set_error(CSPD_E_SHAPE, "P %lld, N %d (1..%d), T %d, kstride %d", (long long)p, n, NMAX, t_atoms,
                             kstride);
        if (p * (int64_t)kstride >= ((int64_t)1 << 31) || p * (int64_t)n >= ((int64_t)1 << 40))
            return set_error(CSPD_E_SHAPE, "too many signals");
        if (p == 0) return CSPD_OK;
        if (!x || !dict || !support || !coef) return set_error(CSPD_E_INVALID, "NULL pointer");
        hipStream_t st = (hipStream_t)hip_stream;
        const int64_t entries = p * kstride;
        // workspace: residual, keys / values twice, counts, offsets, sort and scan storage
        size_t sort_bytes = 0, scan_bytes = 0;
        int *dummy = nullptr;
        int bits = 1;
        while ((1 << bits) <= t_atoms) ++bits;
        if (hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, dummy, dummy, dummy, dummy, (int)entries, 0, bits,
                                               st) != hipSuccess ||
            hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, dummy, dummy, t_atoms, st) != hipSuccess)
            return set_error(CSPD_E_DEVICE, "temporary storage query failed");
        auto al = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t o_r = 0;
        const size_t o_k0 = o_r + al(sizeof(float) * (size_t)(p * n));
        const size_t o_v0 = o_k0 + al(sizeof(int) * (size_t)entries);
        const size_t o_k1 = o_v0 + al(sizeof(int) * (size_t)entries);
        const size_t o_v1 = o_k1 + al(sizeof(int) * (size_t)entries);
        const size_t o_cnt = o_v1 + al(sizeof(int) * (size_t)entries);
        const size_t o_off = o_cnt + al(sizeof(int) * (size_t)t_atoms);
        const size_t o_part = o_off + al(sizeof(int) * (size_t)t_atoms);
        const size_t o_tab = o_part + al(sizeof(double) * (size_t)PG * NUT);
        const size_t o_dold = o_tab + al(sizeof(int) * (size_t)NUT);
        const size_t o_tmp = o_dold + al(sizeof(float) * (size_t)NMAX);
        const size_t total = o_tmp + al(sort_bytes > scan_bytes ? sort_bytes : scan_bytes);
        char *ws = nullptr;
        if (hipMallocAsync((void **)&ws, total, st) != hipSuccess) return set_error(CSPD_E_NOMEM, "workspace");
        float *r = (float *)(ws + o_r);
        int *k0 = (int *)(ws + o_k0), *v0 = (int *)(ws + o_v0), *k1 = (int *)(ws + o_k1), *v1 = (int *)(ws + o_v1);
        int *cnt = (int *)(ws + o_cnt), *off = (int *)(ws + o_off);
        void *tmp = ws + o_tmp;
        double *part = (double *)(ws + o_part);
        int *tab = (int *)(ws + o_tab);
        float *dold = (float *)(ws + o_dold);
        cspd_status rc = CSPD_OK;
        ProfileToken *tok = profile_begin("ksvd_update", st);
        const int bs = 256;
        hipLaunchKernelGGL(k_residual, dim3((unsigned)((p * n + bs - 1) / bs)), dim3(bs), 0, st, x, dict, support, coef,
                           kstride, p, n, r);
        // counts start at zero: a fill kernel rather than a memset (graph-safe)
        hipLaunchKernelGGL(k_fill_zero_i32, dim3((unsigned)((t_atoms + bs - 1) / bs)), dim3(bs), 0, st, cnt, t_atoms);
        hipLaunchKernelGGL(k_keys, dim3((unsigned)((entries + bs - 1) / bs)), dim3(bs), 0, st, support, entries,
                           t_atoms, k0, v0, cnt);
        size_t sb = sort_bytes, cb = scan_bytes;
        if (hipcub::DeviceRadixSort::SortPairs(tmp, sb, k0, k1, v0, v1, (int)entries, 0, bits, st) != hipSuccess ||
            hipcub::DeviceScan::ExclusiveSum(tmp, cb, cnt, off, t_atoms, st) != hipSuccess)
            rc = set_error(CSPD_E_DEVICE, "sort / scan failed");
        if (rc == CSPD_OK) {
            hipLaunchKernelGGL(k_tri_table, dim3(1), dim3(NMAX), 0, st, n, tab);
            for (int k = 0; k < t_atoms; ++k) {
                hipLaunchKernelGGL(k_atom_gram, dim3(PG), dim3(BS), 0, st, k, n, kstride, off, cnt, v1, dict, coef, r,
                                   tab, part);
                hipLaunchKernelGGL(k_atom, dim3(1), dim3(BS), 0, st, k, n, cnt, dict, dold, part, tab, 2000, 1e-12);
                hipLaunchKernelGGL(k_atom_users, dim3(PG), dim3(BS), 0, st, k, n, kstride, off, cnt, v1, dict, dold,
                                   coef, r);
            }
            if (hipGetLastError() != hipSuccess) rc = set_error(CSPD_E_DEVICE, "atom update launch failed");
        }
        profile_end(tok, st);
        (void)hipFreeAsync(ws, st);
        return rc;
    });
}

}  // extern "C"
