// Internal declarations shared by the cspd HIP sources (not installed).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <mutex>
#include <string>

#include "cspd.h"

namespace cspd {

// Largest sparsity per scale the per-patch kernels keep state for.
constexpr int kMaxK = 16;
// full search in coefficient coordinates (Gram matrix precomputed): atoms and
// sparsity it supports; plans with k_max above kMaxK run only this path
constexpr int kMaxBatchAtoms = 8192;
constexpr int kMaxKBatch = 64;
// Per-patch Gram tables are precomputed for shared operators up to this size.
constexpr int kMaxGramAtoms = 1024;
// Candidate vectors longer than kMaxShortLen coordinates (up to kMaxLongLen)
// run on the long-vector kernel, which scores up to kMaxLongCand candidates.
constexpr int kMaxShortLen = 256;
constexpr int kMaxLongLen = 2048;
constexpr int kMaxLongCand = 1024;
// Wavefronts per workgroup of the per-patch kernels (the matrix-core Gram
// kernels use one; see waves_per_block).
constexpr int kWavesPerBlock = 4;

cspd_status set_error(cspd_status code, const char *fmt, ...);

// Runs an entry point's body and turns any C++ exception into a status (and
// the thread's error message), so that nothing thrown inside the library
// crosses the C ABI.
template <typename F>
cspd_status guarded(F &&body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return set_error(CSPD_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return set_error(CSPD_E_DEVICE, "C++ exception: %s", e.what());
    } catch (...) {
        return set_error(CSPD_E_DEVICE, "unknown C++ exception");
    }
}
void clear_error();
bool has_error();
// Resolves this device's address of the no-allocation entry point's static
// workspace (once per device; the device must be current).
void noalloc_setup(int device);

#define CSPD_HIP_CHECK(expr)                                                        \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return ::cspd::set_error(CSPD_E_DEVICE, "%s failed: %s (%s:%d)", #expr,  \
                                     hipGetErrorString(e_), __FILE__, __LINE__);    \
    } while (0)

// How the kernel forms the candidate vectors of one scale.
//  kFold  : identity or mask operator; candidates are D_s columns in the
//           scale's own coordinates, weighted per patch by the square root of
//           the number of observed fine samples in each block (the Gram of
//           Phi U D_s restricted to the block structure), so that plain dot
//           products of the weighted vectors equal those of Phi U D_s.
//  kDense : shared dense operator; candidates are the columns of
//           A_s = Phi U D_s, precomputed by the plan.
enum FoldKind { kFold = 0, kDense = 1 };

struct ScalePlan {
    int n_s = 0;         // signal dimension at this scale
    int t = 0;           // atoms
    int q = 1;           // children per parent atom (1 at scale 0)
    int l = 0;           // candidate vector length (N_s folded, M dense)
    int lp = 0;          // padded row stride of `v` (multiple of 4)
    int fold = kFold;
    void *v = nullptr;        // t x lp, atom-contiguous, zero padded, plan dtype
    void *v_lo = nullptr;     // t x lp, 16-bit copy for the reduced-precision proxy (or null)
    void *nu2 = nullptr;      // t per operator, squared effective norms (null for mask plans)
    void *inv_nu = nullptr;   // t per operator, FP32 reciprocal effective norms (null for mask plans)
    void *gram = nullptr;     // t x t effective Gram (null unless precomputed)
    int *blk_off = nullptr;   // l + 1 (fold only): fine samples of each coarse sample
    int *blk_idx = nullptr;   // N (fold only)
    int blk_ident = 0;        // fold whose blocks are single samples in signal order
    float gsplit = 2048.f;    // power of two: scale of the matrix-core Gram's FP16 split
    // FP16 split of gsplit times v (FP32 plans, scales whose candidates carry
    // weights 0 or 1): per 8 coordinates the four high-part pairs, then the
    // four low-part pairs; t x lp 32-bit words, or null
    void *v_split = nullptr;
    int64_t phase_stride = 0; // elements of v (and words of v_split) per operator phase
};

}  // namespace cspd

namespace cspd {
// A kernel variant for one scale (autotuned or chosen by shape rules).
enum ChoiceKind {
    kChoiceAuto = 0, kChoiceFirstMfma = 1, kChoiceVec = 2, kChoiceGram = 3, kChoiceMfmaGram = 4, kChoiceGemmGram = 5
};
struct KernelChoice {
    int kind = kChoiceAuto;
    int nc = 1;
    int ppw = 1;
    int cand = 0;   // candidate count it was timed on; used only for that count
};
}  // namespace cspd

struct cspd_plan_s {
    int s = 0;           // scales
    int n = 0;           // finest dimension
    int m = 0;           // measurement dimension
    int phi_kind = 0;
    int dtype = 0;
    int corr_mode = 0;
    int rescore_m = 8;
    int k_max = 0;
    int device = 0;
    int n_phases = 1;         // dense operators (per-patch choice when > 1)
    int64_t bytes = 0;
    cspd::ScalePlan sc[CSPD_MAX_SCALES];
    void *d_high = nullptr;   // T_high x N atom-contiguous (plan dtype), for x-hat
    // full search over large dictionaries (FP32 plans, shared operator):
    // the finest effective dictionary in FP64 (T x l, atom-contiguous) and its
    // Gram matrix A^T A (T x T, FP32); null unless built
    void *bat_a64 = nullptr;
    void *bat_g = nullptr;
    // autotuned kernel per scale and sparsity bucket (K <= 4, <= 8, <= 16)
    cspd::KernelChoice tuned[CSPD_MAX_SCALES][3];
    mutable std::mutex mu;   // guards tuned
};

namespace cspd {

// Arguments of one per-patch OMP pass over one scale (a launch).
struct ScaleArgs {
    int64_t b;                  // patches
    const void *y;              // b x y_stride
    int y_stride;
    const uint8_t *mask;        // b x n or null
    int n;                      // finest dimension
    const void *v;              // candidate vectors (t x lp)
    const void *gram;           // t x t (gram mode)
    int t;                      // atoms at this scale
    int l;                      // candidate vector length
    int lp;                     // row stride of v
    int fold;                   // FoldKind
    int m_dense;                // measurement dim when dense (rank bound)
    const int *blk_off;
    const int *blk_idx;
    int blk_ident;              // 1: coordinate t of the scale is fine sample t
    int first;                  // 1: every atom is a candidate
    const int *prev_sup;        // b x prev_stride (first == 0)
    int prev_stride;
    int prev_count;             // entries of the previous scale in each prev_sup row
    const int *prev_kused;      // b
    int q;                      // children per parent
    unsigned qmagic;            // ceil(2^32 / q) for q > 1 (division by q as a high multiply)
    const int *kvec;            // b or null
    int kuni;                   // uniform k
    int last;                   // 1: write coefficients / x-hat
    int scale;                  // scale index (labels only)
    int *sup_out;               // row-major, row stride sup_stride
    int sup_stride;
    int sup_count;              // entries written per row (and the cap on k)
    int *kused_out;             // b
    void *coef_out;             // b x sup_stride (last)
    void *xhat;                 // b x n (last, may be null)
    const void *d_high;         // T_high x n (last)
    const void *hpre;           // b x t correlations with y (gram mode, first scale), or null;
                                // for launch_choice: the workspace the GEMM variant writes them to
    const void *nu2;            // t squared effective norms (with hpre)
    float gsplit;               // power of two: candidates times it fit FP16 (split Gram)
    const void *vsplit;         // t x lp 32-bit words: the candidates split at plan time, or null
    // per-patch operator (plans with several dense operators): phase[b] picks
    // the slice phase[b] * phase_stride of v (and vsplit); a phase outside
    // [0, n_phases) leaves the patch unsolved.  Null: every patch uses slice 0.
    const int *phase;
    int n_phases;
    int64_t phase_stride;
    // reduced-precision first-scale correlations (cross-scale, dense
    // operator): the 16-bit copy of v for the contraction, its format
    // (CSPD_CORR_*), and how many candidates the kernel may re-score in FP32
    // before each pick (0: the correlations are FP32 and no re-scoring runs)
    const void *vlo;
    int corr_lo;
    int hre;
};

// Kernel variants that can run one scale (FP32): the first-scale MFMA kernel,
// the MFMA-Gram kernel, the register shapes and the Gram-table kernel that
// hold `max_cand` candidates.  Returns how many were written (at most cap).
int scale_choices(int dtype, const ScaleArgs &a, int max_cand, bool has_gram, KernelChoice *out, int cap);
// Launches one scale with an explicit variant.
cspd_status launch_choice(int dtype, const ScaleArgs &a, const KernelChoice &c, hipStream_t stream);
// Sparsity bucket of a scale's launch (0: K <= 4, 1: <= 8, 2: <= 16).
int k_bucket(const ScaleArgs &a);

// Selects and launches the per-scale kernel; returns CSPD_E_UNSUPPORTED when
// no instantiation fits.
cspd_status launch_scale(int dtype, const ScaleArgs &a, int max_candidates, bool gram_mode,
                         hipStream_t stream);

// First scale of a cross-scale call on the matrix cores (shared dictionary,
// 16 patches per wavefront); CSPD_E_UNSUPPORTED when the shape does not fit.
// Cross-scale call on a caller-provided workspace (no allocation), and the
// bytes it needs.
size_t cross_call_workspace(const cspd_plan_s *p, int64_t B, const int32_t *k_scale, bool caller_keeps_supports);
cspd_status cross_scale_on(cspd_plan_s *p, int64_t B, const void *y, const uint8_t *mask, const int32_t *k_scale,
                           const int32_t *k_fine, int32_t k_fine_uniform, int32_t *support, void *coef,
                           int32_t *k_used, void *xhat, int32_t *support_coarse, void *work, size_t work_bytes,
                           hipStream_t stream);
// Device bytes per patch of a cross-scale call's own workspace (beyond the
// caller's buffers and the coarse supports).
int64_t cross_workspace_per_patch(const cspd_plan_s *p);
// Batched first-scale correlations H = Y A_0 (b x t, FP32) of a shared dense
// operator on the matrix cores, and whether a scale qualifies.
bool proxy_gemm_fits(int dtype, const ScaleArgs &a);
cspd_status launch_proxy_gemm(int dtype, const ScaleArgs &a, float *h, hipStream_t stream);
// With several operators (a.phase) the GEMM groups the patches by operator
// first: each operator's first position and first tile (P + 1 entries),
// and the patch indices listed operator by operator.  The workspace starts
// phase_groups_offset bytes after the b x t correlations and holds
// phase_groups_bytes.
struct PhaseGroups {
    int *seg;
    int *tile;
    int *perm;
};
size_t phase_groups_offset(int64_t B, int t);
size_t phase_groups_bytes(int64_t B, int P);
PhaseGroups phase_groups(void *base, int64_t B, int P);
// Long-vector kernel (one workgroup per patch, FP64 least squares): whether
// it can run a scale with this many candidates, and its launch.
bool long_fits(const ScaleArgs &a, int max_cand);
cspd_status launch_long(int dtype, const ScaleArgs &a, int max_cand, hipStream_t stream);
// Whether the first-scale matrix-core kernel has an instance for this scale.
bool first_mfma_fits(int dtype, const ScaleArgs &a);
cspd_status launch_first_mfma(int dtype, const ScaleArgs &a, hipStream_t stream);

// Full-dictionary proxy on matrix cores (large T).
cspd_status launch_full_mfma(const cspd_plan_s *p, int64_t b, const void *y, const uint8_t *mask,
                             const int *kvec, int kuni, int *support, void *coef, int *k_used,
                             void *xhat, hipStream_t stream);

// Optional per-launch event timing (cspd_profile_enable).  Returns a token
// to pass to profile_end after the launch; null when recording is off.
struct ProfileToken;
ProfileToken *profile_begin(const char *label, hipStream_t stream);
void profile_end(ProfileToken *tok, hipStream_t stream);
// The same for a launch that records the token's events itself (the
// dispatch's own start and end timestamps, no extra packets on the stream):
// profile_open gives the events to pass to hipExtLaunchKernel, profile_close
// files the token.
ProfileToken *profile_open(const char *label, hipEvent_t *start, hipEvent_t *stop);
void profile_close(ProfileToken *tok);

// Launches a kernel on `stream`, timed by profile_open / profile_close when
// recording is on (the kernel's own dispatch records the events).
template <typename K, typename... Args>
inline void launch_timed(const char *label, K kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t stream,
                         Args... args)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ProfileToken *tok = profile_open(label, &e0, &e1);
    if (tok) {
        hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, e0, e1, 0, args...);
        profile_close(tok);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, stream, args...);
    }
}
// While alive, this thread's launches record no profiling events (graph capture).
struct ProfileSuspend {
    ProfileSuspend();
    ~ProfileSuspend();
};

// Plan-time kernels.
cspd_status plan_effective(cspd_plan_s *p, const cspd_plan_desc *d, hipStream_t stream);

// Plain library GEMM (rocBLAS, FP64): column-major C (m x n) = A^T B with A
// stored k x m (leading dimension lda) and B stored k x n, on `st`.
cspd_status gemm_tn_f64(int device, hipStream_t st, int m, int n, int k, const double *a, int lda,
                        const double *b, int ldb, double *c, int ldc);
// Search in coefficient coordinates over the plan's finest scale (its Gram
// matrix precomputed): whether the plan has the tables, and the launch.
bool batch_fits(const cspd_plan_s *p);
// With a.first == 0 it runs zero-tree OMP's finest scale over the children of
// the coarse support (at most max_cand candidates).
cspd_status launch_batch(const cspd_plan_s *p, const ScaleArgs &a, int max_cand, hipStream_t st);

}  // namespace cspd
