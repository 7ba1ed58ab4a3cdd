// C-ABI entry points: argument validation, plan construction and dispatch of
// the per-scale kernels.  Validation happens before any HIP call.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cspd_internal.h"

namespace cspd {

// Message of the last error on this thread: a fixed buffer, so that setting
// it neither allocates nor throws.
static thread_local char g_err[512];

cspd_status set_error(cspd_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

bool has_error() { return g_err[0] != 0; }

bool scale_vec_fits(int lp, int max_cand, bool f64);

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

cspd_status validate_desc(const cspd_plan_desc *d)
{
    if (!d) return set_error(CSPD_E_INVALID, "desc is NULL");
    const int S = d->n_scales;
    if (S < 1 || S > CSPD_MAX_SCALES) return set_error(CSPD_E_INVALID, "n_scales %d outside 1..%d", S, CSPD_MAX_SCALES);
    for (int s = 0; s < S; ++s) {
        if (d->dim[s] <= 0 || d->atoms[s] <= 0)
            return set_error(CSPD_E_SHAPE, "scale %d: dim %d atoms %d must be positive", s, d->dim[s], d->atoms[s]);
        if (!d->dict[s]) return set_error(CSPD_E_INVALID, "dict[%d] is NULL", s);
        if (s > 0 && d->atoms[s] % d->atoms[s - 1] != 0)
            return set_error(CSPD_E_SHAPE, "atoms[%d] = %d is not a multiple of atoms[%d] = %d", s,
                             d->atoms[s], s - 1, d->atoms[s - 1]);
        // the kernels divide candidate indices by q with a 32-bit high multiply
        if (s > 0 && d->atoms[s] / d->atoms[s - 1] >= (1 << 22))
            return set_error(CSPD_E_SHAPE, "scale %d: %d children per atom (at most 2^22 - 1)", s,
                             d->atoms[s] / d->atoms[s - 1]);
        // kernels index a dictionary with 32-bit offsets (rows padded to at
        // most twice the length, and at least the measurement dimension)
        const int64_t len = 2 * (int64_t)(d->dim[s] > d->m ? d->dim[s] : d->m) + 16;
        if ((int64_t)d->atoms[s] * len >= ((int64_t)1 << 31))
            return set_error(CSPD_E_SHAPE, "scale %d: %d atoms of length %d exceed 2^31 elements", s, d->atoms[s],
                             d->dim[s]);
    }
    for (int s = 0; s + 1 < S; ++s) {
        if (!d->up_map[s]) return set_error(CSPD_E_INVALID, "up_map[%d] is NULL", s);
        std::vector<char> seen(d->dim[s], 0);
        for (int j = 0; j < d->dim[s + 1]; ++j) {
            const int v = d->up_map[s][j];
            if (v < 0 || v >= d->dim[s])
                return set_error(CSPD_E_SHAPE, "up_map[%d][%d] = %d outside [0, %d)", s, j, v, d->dim[s]);
            seen[v] = 1;
        }
        for (int t = 0; t < d->dim[s]; ++t)
            if (!seen[t]) return set_error(CSPD_E_SHAPE, "up_map[%d] does not reach coarse sample %d", s, t);
    }
    const int N = d->dim[S - 1];
    if (d->phi_kind != CSPD_PHI_IDENTITY && d->phi_kind != CSPD_PHI_DENSE && d->phi_kind != CSPD_PHI_MASK)
        return set_error(CSPD_E_INVALID, "phi_kind %d unknown", d->phi_kind);
    if (d->phi_kind == CSPD_PHI_DENSE) {
        if (!d->phi) return set_error(CSPD_E_INVALID, "dense phi is NULL");
        if (d->m <= 0) return set_error(CSPD_E_SHAPE, "m = %d must be positive", d->m);
    } else if (d->m != N) {
        return set_error(CSPD_E_SHAPE, "m = %d must equal N = %d for this phi_kind", d->m, N);
    }
    if (d->dtype != CSPD_F32 && d->dtype != CSPD_F64) return set_error(CSPD_E_INVALID, "dtype %d unknown", d->dtype);
    if (d->corr_mode < CSPD_CORR_NATIVE || d->corr_mode > CSPD_CORR_F16_RESCORE)
        return set_error(CSPD_E_INVALID, "corr_mode %d unknown", d->corr_mode);
    if (d->corr_mode != CSPD_CORR_NATIVE && d->dtype != CSPD_F32)
        return set_error(CSPD_E_INVALID, "reduced-precision proxy needs an FP32 plan");
    if (d->rescore_m < 0 || d->rescore_m > 16) return set_error(CSPD_E_INVALID, "rescore_m %d outside 0..16", d->rescore_m);
    if (d->k_max < 1) return set_error(CSPD_E_SHAPE, "k_max %d must be >= 1", d->k_max);
    if (d->k_max > kMaxKBatch)
        return set_error(CSPD_E_UNSUPPORTED, "k_max %d above the supported %d", d->k_max, kMaxKBatch);
    if (d->k_max > kMaxK && (d->dtype != CSPD_F32 || d->phi_kind == CSPD_PHI_MASK || d->n_phases > 1))
        return set_error(CSPD_E_UNSUPPORTED,
                         "k_max %d above %d needs the FP32 full search over a shared operator", d->k_max, kMaxK);
    for (int s = 0; s < S; ++s) {
        const int l = d->phi_kind == CSPD_PHI_DENSE ? d->m : d->dim[s];
        const int cap = d->dtype == CSPD_F32 ? kMaxLongLen : kMaxShortLen;
        if (l > cap) return set_error(CSPD_E_UNSUPPORTED, "scale %d: vector length %d above %d", s, l, cap);
    }
    if (d->dim[S - 1] > kMaxLongLen)
        return set_error(CSPD_E_UNSUPPORTED, "signal dimension %d above %d", d->dim[S - 1], kMaxLongLen);
    if (d->device < 0) return set_error(CSPD_E_INVALID, "device %d", d->device);
    if (d->n_phases < 0 || d->n_phases > 4096) return set_error(CSPD_E_INVALID, "n_phases %d outside 0..4096", d->n_phases);
    if (d->n_phases > 1 && d->phi_kind != CSPD_PHI_DENSE)
        return set_error(CSPD_E_INVALID, "several operators (n_phases %d) need CSPD_PHI_DENSE", d->n_phases);
    return CSPD_OK;
}

void free_plan(cspd_plan_s *p)
{
    if (!p) return;
    for (int s = 0; s < CSPD_MAX_SCALES; ++s) {
        ScalePlan &sc = p->sc[s];
        if (sc.v) (void)hipFree(sc.v);
        if (sc.v_lo) (void)hipFree(sc.v_lo);
        if (sc.v_split) (void)hipFree(sc.v_split);
        if (sc.nu2) (void)hipFree(sc.nu2);
        if (sc.inv_nu) (void)hipFree(sc.inv_nu);
        if (sc.gram) (void)hipFree(sc.gram);
        if (sc.blk_off) (void)hipFree(sc.blk_off);
        if (sc.blk_idx) (void)hipFree(sc.blk_idx);
    }
    if (p->d_high) (void)hipFree(p->d_high);
    if (p->bat_a64) (void)hipFree(p->bat_a64);
    if (p->bat_g) (void)hipFree(p->bat_g);
    delete p;
}

size_t elem_size(const cspd_plan_s *p) { return p->dtype == CSPD_F64 ? sizeof(double) : sizeof(float); }

// The calls take their workspace from the device's default stream-ordered
// pool (hipMallocAsync) and give it back at the end of the call.  By default
// the pool returns freed memory to the device at once, so every call would
// map its workspace afresh; a release threshold of kPoolKeepBytes keeps up
// to that much freed memory in the pool between calls.  Set once per device
// at the first plan on it, and only raised, never lowered.
constexpr uint64_t kPoolKeepBytes = (uint64_t)2 << 30;

void keep_workspace_pool(int device)
{
    static std::mutex mu;
    static bool done[64] = {};
    std::lock_guard<std::mutex> g(mu);
    if (device < 0 || device >= 64 || done[device]) return;
    done[device] = true;
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, device) != hipSuccess || !pool) return;
    uint64_t cur = 0;
    if (hipMemPoolGetAttribute(pool, hipMemPoolAttrReleaseThreshold, &cur) == hipSuccess && cur >= kPoolKeepBytes)
        return;
    uint64_t thr = kPoolKeepBytes;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
}

// Arguments common to every scale of one call.
ScaleArgs base_args(const cspd_plan_s *p, int s, int64_t B, const void *y, const uint8_t *mask)
{
    const ScalePlan &sc = p->sc[s];
    ScaleArgs a{};
    a.b = B;
    a.y = y;
    a.y_stride = p->m;
    a.mask = p->phi_kind == CSPD_PHI_MASK ? mask : nullptr;
    a.n = p->n;
    a.v = sc.v;
    a.gram = sc.gram;
    a.t = sc.t;
    a.l = sc.l;
    a.lp = sc.lp;
    a.fold = sc.fold;
    a.m_dense = p->m;
    a.blk_off = sc.blk_off;
    a.blk_idx = sc.blk_idx;
    a.blk_ident = sc.blk_ident;
    a.gsplit = sc.gsplit;
    a.vsplit = sc.v_split;
    a.phase = nullptr;
    a.n_phases = p->n_phases;
    a.phase_stride = sc.phase_stride;
    a.q = sc.q;
    a.qmagic = sc.q > 1 ? (unsigned)((((uint64_t)1 << 32) + (uint64_t)sc.q - 1) / (uint64_t)sc.q) : 0u;
    a.d_high = p->d_high;
    if (s == 0 && p->s >= 2 && p->corr_mode != CSPD_CORR_NATIVE && sc.v_lo) {
        a.vlo = sc.v_lo;
        a.corr_lo = p->corr_mode;
        a.hre = p->rescore_m;
    }
    return a;
}

// Largest candidate count of scale s when it is searched in full (first) or
// restricted to the children of k_prev atoms.
int max_candidates(const cspd_plan_s *p, int s, bool first, int k_prev)
{
    if (first) return p->sc[s].t;
    const long v = (long)p->sc[s].q * k_prev;
    return (int)(v < p->sc[s].t ? v : p->sc[s].t);
}


// Validated scalars of one cross-scale call.
struct CrossCall {
    const int32_t *phase = nullptr;   // per-patch operator (plans with several)
    int ksum = 0;
    int cand[CSPD_MAX_SCALES] = {};
    char gram[CSPD_MAX_SCALES] = {};
    char lng[CSPD_MAX_SCALES] = {};   // 1: the long-vector kernel; 2: coefficient coordinates
};

cspd_status prepare_cross(const cspd_plan_s *p, int64_t B, const void *y, const uint8_t *mask,
                          const int32_t *k_scale, const int32_t *k_fine, int32_t k_fine_uniform,
                          const int32_t *support, const void *coef, const int32_t *k_used, CrossCall &c)
{
    if (B < 0) return set_error(CSPD_E_INVALID, "B = %lld", (long long)B);
    if (!k_scale) return set_error(CSPD_E_INVALID, "k_scale is NULL");
    if (p->k_max > kMaxK && p->s > 1)
        return set_error(CSPD_E_UNSUPPORTED, "a plan with k_max %d above %d runs full OMP only", p->k_max, kMaxK);
    c.ksum = 0;
    for (int s = 0; s + 1 < p->s; ++s) {
        if (k_scale[s] < 0 || k_scale[s] > p->k_max)
            return set_error(CSPD_E_SHAPE, "k_scale[%d] = %d outside [0, k_max = %d]", s, k_scale[s], p->k_max);
        c.ksum += k_scale[s];
    }
    if (!k_fine && (k_fine_uniform < 0 || k_fine_uniform > p->k_max))
        return set_error(CSPD_E_SHAPE, "k_fine_uniform %d outside [0, k_max = %d]", k_fine_uniform, p->k_max);
    if (B == 0) return CSPD_OK;
    if (!y || !support || !coef || !k_used) return set_error(CSPD_E_INVALID, "y / support / coef / k_used is NULL");
    if (p->phi_kind == CSPD_PHI_MASK && !mask) return set_error(CSPD_E_INVALID, "mask plan needs a mask");
    // candidate counts per scale must have kernels before anything is launched
    for (int s = 0; s < p->s; ++s) {
        const int kprev = s == 0 ? 0 : k_scale[s - 1];
        c.cand[s] = max_candidates(p, s, s == 0, kprev);
        const bool short_ok = scale_vec_fits(p->sc[s].lp, c.cand[s], p->dtype == CSPD_F64) ||
                              (s == 0 && p->sc[s].gram);
        if (s == p->s - 1 && s > 0 && p->sc[s].lp > kMaxShortLen && batch_fits(p) &&
            c.cand[s] <= kMaxBatchAtoms) {
            c.lng[s] = 2;   // zero-tree finest scale in coefficient coordinates (Gram table)
        } else if (p->sc[s].lp > kMaxShortLen || !short_ok) {
            ScaleArgs la = base_args(p, s, B, y, mask);
            if (p->dtype != CSPD_F32 || !long_fits(la, c.cand[s]))
                return set_error(CSPD_E_UNSUPPORTED, "scale %d: no long-vector kernel for %d candidates of length %d",
                                 s, c.cand[s], p->sc[s].l);
            c.lng[s] = 1;
        } else if (!scale_vec_fits(p->sc[s].lp, c.cand[s], p->dtype == CSPD_F64)) {
            if (s == 0 && p->sc[s].gram) c.gram[s] = 1;
            else return set_error(CSPD_E_UNSUPPORTED, "scale %d: no kernel for %d candidates of length %d",
                                  s, c.cand[s], p->sc[s].l);
        }
    }
    return CSPD_OK;
}

// Whether scale 0 runs as a batched GEMM of its correlations followed by the
// Gram-table kernel (shared dense operator, FP32, precomputed Gram and norms).
bool first_gemm_path(const cspd_plan_s *p)
{
    const ScalePlan &sc = p->sc[0];
    int nc = 1;
    while (nc * 64 < sc.t) nc *= 2;
    return p->dtype == CSPD_F32 && p->s >= 2 && sc.fold == kDense && sc.gram && sc.nu2 && sc.lp >= 16 &&
           sc.lp <= 128 && sc.l == p->m && nc <= 16;
}

// Workspace of a cross-scale call: the coarse scales' k_used, their supports
// unless the caller keeps them, and scale 0's correlations on the GEMM path.
size_t hpre_offset(const cspd_plan_s *p, int64_t B, int ksum, bool caller_keeps_supports)
{
    const int64_t nk = B * (p->s - 1);
    const size_t ints = sizeof(int32_t) * (size_t)(nk + (caller_keeps_supports ? 0 : B * (int64_t)ksum));
    return (ints + 255) / 256 * 256;
}

size_t cross_workspace_bytes(const cspd_plan_s *p, int64_t B, int ksum, bool caller_keeps_supports)
{
    const size_t off = hpre_offset(p, B, ksum, caller_keeps_supports);
    if (!first_gemm_path(p)) return off;
    // the correlations, then (several operators) the grouping of the patches
    return off + (p->n_phases > 1 ? phase_groups_offset(B, p->sc[0].t) + phase_groups_bytes(B, p->n_phases)
                                  : sizeof(float) * (size_t)B * (size_t)p->sc[0].t);
}

// Arguments of scale s of a cross-scale call.
ScaleArgs cross_scale_args(const cspd_plan_s *p, int s, int64_t B, const void *y, const uint8_t *mask,
                           const int32_t *k_scale, const int32_t *k_fine, int32_t k_fine_uniform,
                           int32_t *support, void *coef, int32_t *k_used, void *xhat, int32_t *coarse,
                           int32_t *kused_c, int ksum)
{
    int off = 0;
    for (int i = 0; i < s; ++i) off += k_scale[i];
    ScaleArgs a = base_args(p, s, B, y, mask);
    a.first = s == 0;
    a.scale = s;
    if (s > 0) {
        a.prev_sup = coarse + (off - k_scale[s - 1]);
        a.prev_stride = ksum;
        a.prev_count = k_scale[s - 1];
        a.prev_kused = kused_c + B * (s - 1);
    }
    if (s + 1 < p->s) {
        a.kvec = nullptr;
        a.kuni = k_scale[s];
        a.last = 0;
        a.sup_out = coarse + off;
        a.sup_stride = ksum;
        a.sup_count = k_scale[s];
        a.kused_out = kused_c + B * s;
    } else {
        a.kvec = k_fine;
        a.kuni = k_fine_uniform;
        a.last = 1;
        a.sup_out = support;
        a.sup_stride = p->k_max;
        a.sup_count = p->k_max;
        a.kused_out = k_used;
        a.coef_out = coef;
        a.xhat = xhat;
    }
    return a;
}

// One scale with the plan's autotuned kernel if there is one, else by the
// shape rules.  `hpre` is the workspace of scale 0's correlations on the GEMM
// path (else unused).
cspd_status launch_cross_scale(const cspd_plan_s *p, int s, const ScaleArgs &a0, const CrossCall &c, float *hpre,
                               hipStream_t st)
{
    ScaleArgs a = a0;
    if (c.lng[s] == 2) return launch_batch(p, a, c.cand[s], st);
    if (c.lng[s]) return launch_long(p->dtype, a, c.cand[s], st);
    if (s == 0 && first_gemm_path(p)) {
        a.hpre = hpre;   // workspace for the GEMM variant
        a.nu2 = p->sc[0].nu2;
    }
    KernelChoice tc;
    if (p->n_phases == 1) {
        std::lock_guard<std::mutex> lk(p->mu);
        tc = p->tuned[s][k_bucket(a)];
    }
    if (tc.kind != kChoiceAuto && tc.cand == c.cand[s]) {
        const cspd_status rc = launch_choice(p->dtype, a, tc, st);
        if (rc == CSPD_E_UNSUPPORTED && !has_error())
            return set_error(rc, "scale %d: tuned kernel kind %d (nc %d, ppw %d) cannot run this call", s, tc.kind,
                             tc.nc, tc.ppw);
        return rc;
    }
    if (s == 0 && first_gemm_path(p)) {
        KernelChoice gg;
        gg.kind = kChoiceGemmGram;
        while (gg.nc * 64 < c.cand[0]) gg.nc *= 2;
        return launch_choice(p->dtype, a, gg, st);
    }
    a.hpre = nullptr;
    // the first-scale matrix-core kernel keeps one shared dictionary
    cspd_status rc = s == 0 && p->n_phases == 1 ? launch_first_mfma(p->dtype, a, st) : CSPD_E_UNSUPPORTED;
    if (rc == CSPD_E_UNSUPPORTED) rc = launch_scale(p->dtype, a, c.cand[s], c.gram[s], st);
    return rc;
}

// One kernel per scale on `st`; `work` holds cross_workspace_bytes.
cspd_status run_cross(const cspd_plan_s *p, int64_t B, const void *y, const uint8_t *mask,
                      const int32_t *k_scale, const int32_t *k_fine, int32_t k_fine_uniform,
                      int32_t *support, void *coef, int32_t *k_used, void *xhat, int32_t *support_coarse,
                      int32_t *work, const CrossCall &c, hipStream_t st)
{
    const int64_t nk = B * (p->s - 1);
    int32_t *kused_c = work;
    int32_t *coarse = support_coarse ? support_coarse : work + nk;
    float *hpre = (float *)((char *)work + hpre_offset(p, B, c.ksum, support_coarse != nullptr));
    cspd_status rc = CSPD_OK;
    for (int s = 0; s < p->s && rc == CSPD_OK; ++s) {
        ScaleArgs a = cross_scale_args(p, s, B, y, mask, k_scale, k_fine, k_fine_uniform, support, coef,
                                             k_used, xhat, coarse, kused_c, c.ksum);
        a.phase = c.phase;
        rc = launch_cross_scale(p, s, a, c, hpre, st);
    }
    return rc;
}

}  // namespace

// A cross-scale call on a workspace the caller provides (the serving loop's
// per-slot buffers): no allocation.  `work` must hold cross_call_workspace
// bytes for the same arguments.
size_t cross_call_workspace(const cspd_plan_s *p, int64_t B, const int32_t *k_scale, bool caller_keeps_supports)
{
    int ksum = 0;
    for (int s = 0; s + 1 < p->s; ++s) ksum += k_scale[s];
    return cross_workspace_bytes(p, B, ksum, caller_keeps_supports);
}

cspd_status cross_scale_on(cspd_plan_s *p, int64_t B, const void *y, const uint8_t *mask, const int32_t *k_scale,
                           const int32_t *k_fine, int32_t k_fine_uniform, int32_t *support, void *coef,
                           int32_t *k_used, void *xhat, int32_t *support_coarse, void *work, size_t work_bytes,
                           hipStream_t st)
{
    clear_error();
    if (p->n_phases > 1 && B > 0)
        return set_error(CSPD_E_INVALID, "plan has %d operators: only cspd_omp_cross_scale_phased runs it", p->n_phases);
    if (p->s == 1) return cspd_omp_full(p, B, y, mask, k_fine, k_fine_uniform, support, coef, k_used, xhat, st);
    CrossCall c;
    cspd_status rc = prepare_cross(p, B, y, mask, k_scale, k_fine, k_fine_uniform, support, coef, k_used, c);
    if (rc != CSPD_OK || B == 0) return rc;
    if (work_bytes < cross_workspace_bytes(p, B, c.ksum, support_coarse != nullptr))
        return set_error(CSPD_E_INVALID, "workspace of %zu bytes is too small", work_bytes);
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(CSPD_E_DEVICE, "hipSetDevice(%d) failed", p->device);
    return run_cross(p, B, y, mask, k_scale, k_fine, k_fine_uniform, support, coef, k_used, xhat, support_coarse,
                     (int32_t *)work, c, st);
}

int64_t cross_workspace_per_patch(const cspd_plan_s *p)
{
    int64_t per = (int64_t)sizeof(int32_t) * (p->s - 1);
    if (first_gemm_path(p)) per += (int64_t)sizeof(float) * p->sc[0].t + (p->n_phases > 1 ? 4 : 0);
    return per;
}
}  // namespace cspd

struct cspd_graph_s {
    int device = 0;
    void *work = nullptr;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace cspd;

extern "C" {

const char *cspd_last_error(void) { return cspd::g_err; }

const char *cspd_version(void) { return "cspd 0.1 (gfx950)"; }

cspd_status cspd_plan(const cspd_plan_desc *d, cspd_plan_t *out)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!out) return set_error(CSPD_E_INVALID, "out is NULL");
        *out = nullptr;
        cspd_status rc = validate_desc(d);
        if (rc != CSPD_OK) return rc;
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
            return set_error(CSPD_E_DEVICE, "no HIP device available");
        if (d->device >= ndev) return set_error(CSPD_E_INVALID, "device %d of %d", d->device, ndev);
        DeviceGuard g(d->device);
        if (!g.ok) return set_error(CSPD_E_DEVICE, "hipSetDevice(%d) failed", d->device);
        noalloc_setup(d->device);
        keep_workspace_pool(d->device);
        cspd_plan_s *p = new (std::nothrow) cspd_plan_s();
        if (!p) return set_error(CSPD_E_NOMEM, "host allocation failed");
        p->s = d->n_scales;
        p->n = d->dim[d->n_scales - 1];
        p->m = d->m;
        p->phi_kind = d->phi_kind;
        p->dtype = d->dtype;
        p->corr_mode = d->corr_mode;
        p->rescore_m = d->rescore_m ? d->rescore_m : 8;
        p->k_max = d->k_max;
        p->n_phases = d->n_phases > 1 ? d->n_phases : 1;
        p->device = d->device;
        hipStream_t st;
        if (hipStreamCreate(&st) != hipSuccess) {
            free_plan(p);
            return set_error(CSPD_E_DEVICE, "hipStreamCreate failed");
        }
        rc = plan_effective(p, d, st);
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
        if (rc != CSPD_OK) {
            free_plan(p);
            return rc;
        }
        *out = p;
        return CSPD_OK;
    });
}

void cspd_plan_destroy(cspd_plan_t p)
{
    try {
        if (!p) return;
        DeviceGuard g(p->device);
        (void)hipDeviceSynchronize();
        free_plan(p);
    } catch (...) {
        // nothing may cross the C ABI; the object is left as it is
    }
}

int64_t cspd_plan_device_bytes(cspd_plan_t p) { return p ? p->bytes : 0; }

}  // extern "C"

namespace cspd {
namespace {

// Algorithm 1 over the finest dictionary; `phase` picks each patch's operator
// on plans with several (null: operator 0).
cspd_status full_on(cspd_plan_s *p, int64_t B, const int32_t *phase, const void *y, const uint8_t *mask,
                    const int32_t *k, int32_t k_uniform, int32_t *support, void *coef, int32_t *k_used, void *xhat,
                    hipStream_t st)
{
    if (B < 0) return set_error(CSPD_E_INVALID, "B = %lld", (long long)B);
    if (!k && (k_uniform < 0 || k_uniform > p->k_max))
        return set_error(CSPD_E_SHAPE, "k_uniform %d outside [0, k_max = %d]", k_uniform, p->k_max);
    if (B == 0) return CSPD_OK;
    if (!y || !support || !coef || !k_used) return set_error(CSPD_E_INVALID, "y / support / coef / k_used is NULL");
    if (p->phi_kind == CSPD_PHI_MASK && !mask) return set_error(CSPD_E_INVALID, "mask plan needs a mask");
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(CSPD_E_DEVICE, "hipSetDevice(%d) failed", p->device);
    const int s = p->s - 1;
    const ScalePlan &sc = p->sc[s];
    ScaleArgs a = base_args(p, s, B, y, mask);
    a.phase = phase;
    a.first = 1;
    a.scale = s;
    a.kvec = k;
    a.kuni = k_uniform;
    a.last = 1;
    a.sup_out = support;
    a.sup_stride = p->k_max;
    a.sup_count = p->k_max;
    a.kused_out = k_used;
    a.coef_out = coef;
    a.xhat = xhat;
    const int cand = sc.t;
    cspd_status rc;
    // full search in coefficient coordinates: built for dictionaries (or
    // sparsities) that no per-patch kernel holds
    if (batch_fits(p)) return launch_batch(p, a, sc.t, st);
    if (p->k_max > kMaxK)
        return set_error(CSPD_E_UNSUPPORTED, "k_max %d above %d needs the full-search tables (T = %d)", p->k_max,
                         kMaxK, sc.t);
    if (sc.lp > kMaxShortLen) {
        rc = p->dtype == CSPD_F32 && long_fits(a, cand) ? launch_long(p->dtype, a, cand, st) : CSPD_E_UNSUPPORTED;
        if (rc == CSPD_E_UNSUPPORTED && !has_error())
            return set_error(rc, "no long-vector full search for T = %d (at most %d), length %d", sc.t, kMaxLongCand,
                             sc.l);
        return rc;
    }
    const bool fits = scale_vec_fits(sc.lp, cand, p->dtype == CSPD_F64);
    // a reduced-precision proxy runs on the full-search kernel, which keeps
    // one shared dictionary (not with several operators)
    const bool lowp = p->corr_mode != CSPD_CORR_NATIVE && sc.v_lo != nullptr;
    if ((fits || sc.gram) && !lowp) rc = launch_scale(p->dtype, a, cand, !fits, st);
    else if (p->n_phases == 1) rc = launch_full_mfma(p, B, y, mask, k, k_uniform, support, coef, k_used, xhat, st);
    else rc = CSPD_E_UNSUPPORTED;
    if (rc == CSPD_E_UNSUPPORTED && p->dtype == CSPD_F32 && long_fits(a, cand)) {
        clear_error();
        rc = launch_long(p->dtype, a, cand, st);
    }
    if (rc == CSPD_E_UNSUPPORTED && !has_error())
        return set_error(rc, "no full-search kernel for T = %d, length %d", sc.t, sc.l);
    return rc;
}

// Zero-tree OMP on a stream-ordered temporary workspace.
cspd_status cross_impl(cspd_plan_s *p, int64_t B, const int32_t *phase, const void *y, const uint8_t *mask,
                       const int32_t *k_scale, const int32_t *k_fine, int32_t k_fine_uniform, int32_t *support,
                       void *coef, int32_t *k_used, void *xhat, int32_t *support_coarse, hipStream_t st)
{
    if (p->s == 1) return full_on(p, B, phase, y, mask, k_fine, k_fine_uniform, support, coef, k_used, xhat, st);
    CrossCall c;
    cspd_status rc = prepare_cross(p, B, y, mask, k_scale, k_fine, k_fine_uniform, support, coef, k_used, c);
    if (rc != CSPD_OK || B == 0) return rc;
    c.phase = phase;
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(CSPD_E_DEVICE, "hipSetDevice(%d) failed", p->device);
    // coarse supports: the caller's buffer, or a stream-ordered temporary
    int32_t *work = nullptr;
    const size_t wbytes = cross_workspace_bytes(p, B, c.ksum, support_coarse != nullptr);
    if (hipMallocAsync((void **)&work, wbytes, st) != hipSuccess)
        return set_error(CSPD_E_NOMEM, "workspace of %zu bytes", wbytes);
    rc = run_cross(p, B, y, mask, k_scale, k_fine, k_fine_uniform, support, coef, k_used, xhat, support_coarse, work,
                   c, st);
    (void)hipFreeAsync(work, st);
    return rc;
}

}  // namespace
}  // namespace cspd

extern "C" {

cspd_status cspd_omp_full(cspd_plan_t p, int64_t B, const void *y, const uint8_t *mask,
                          const int32_t *k, int32_t k_uniform, int32_t *support, void *coef,
                          int32_t *k_used, void *xhat, void *hip_stream)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!p) return set_error(CSPD_E_INVALID, "plan is NULL");
        if (p->n_phases > 1 && B > 0)
            return set_error(CSPD_E_INVALID, "plan has %d operators: use cspd_omp_cross_scale_phased", p->n_phases);
        return full_on(p, B, nullptr, y, mask, k, k_uniform, support, coef, k_used, xhat, (hipStream_t)hip_stream);
    });
}

cspd_status cspd_omp_cross_scale_phased(cspd_plan_t p, int64_t B, const int32_t *phase, const void *y,
                                        const uint8_t *mask, const int32_t *k_scale, const int32_t *k_fine,
                                        int32_t k_fine_uniform, int32_t *support, void *coef, int32_t *k_used,
                                        void *xhat, int32_t *support_coarse, void *hip_stream)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!p) return set_error(CSPD_E_INVALID, "plan is NULL");
        if (p->n_phases > 1 && !phase && B > 0)
            return set_error(CSPD_E_INVALID, "plan has %d operators and phase is NULL", p->n_phases);
        return cross_impl(p, B, phase, y, mask, k_scale, k_fine, k_fine_uniform, support, coef, k_used, xhat,
                          support_coarse, (hipStream_t)hip_stream);
    });
}

cspd_status cspd_omp_cross_scale(cspd_plan_t p, int64_t B, const void *y, const uint8_t *mask,
                                 const int32_t *k_scale, const int32_t *k_fine,
                                 int32_t k_fine_uniform, int32_t *support, void *coef,
                                 int32_t *k_used, void *xhat, int32_t *support_coarse,
                                 void *hip_stream)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!p) return set_error(CSPD_E_INVALID, "plan is NULL");
        if (p->n_phases > 1 && B > 0)
            return set_error(CSPD_E_INVALID, "plan has %d operators: use cspd_omp_cross_scale_phased", p->n_phases);
        return cross_impl(p, B, nullptr, y, mask, k_scale, k_fine, k_fine_uniform, support, coef, k_used, xhat,
                          support_coarse, (hipStream_t)hip_stream);
    });
}

cspd_status cspd_graph_cross_scale(cspd_plan_t p, int64_t B, const void *y, const uint8_t *mask,
                                   const int32_t *k_scale, const int32_t *k_fine,
                                   int32_t k_fine_uniform, int32_t *support, void *coef,
                                   int32_t *k_used, void *xhat, int32_t *support_coarse,
                                   cspd_graph_t *out)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!out) return set_error(CSPD_E_INVALID, "out is NULL");
        *out = nullptr;
        if (!p) return set_error(CSPD_E_INVALID, "plan is NULL");
        if (B <= 0) return set_error(CSPD_E_INVALID, "B = %lld (a graph needs patches)", (long long)B);
        if (p->n_phases > 1)
            return set_error(CSPD_E_INVALID, "plan has %d operators: only cspd_omp_cross_scale_phased runs it", p->n_phases);
        CrossCall c;
        if (p->s > 1) {
            const cspd_status rc = prepare_cross(p, B, y, mask, k_scale, k_fine, k_fine_uniform, support, coef,
                                                 k_used, c);
            if (rc != CSPD_OK) return rc;
        }
        DeviceGuard g(p->device);
        if (!g.ok) return set_error(CSPD_E_DEVICE, "hipSetDevice(%d) failed", p->device);
        cspd_graph_s *gr = new (std::nothrow) cspd_graph_s();
        if (!gr) return set_error(CSPD_E_NOMEM, "host allocation failed");
        gr->device = p->device;
        auto fail = [&](cspd_status code, const char *what) {
            cspd_graph_destroy(gr);
            return set_error(code, "%s", what);
        };
        const size_t wbytes = p->s > 1 ? cross_workspace_bytes(p, B, c.ksum, support_coarse != nullptr) : 0;
        if (wbytes && hipMalloc(&gr->work, wbytes) != hipSuccess) return fail(CSPD_E_NOMEM, "graph workspace");
        if (hipStreamCreateWithFlags(&gr->capture, hipStreamNonBlocking) != hipSuccess)
            return fail(CSPD_E_DEVICE, "capture stream");
        if (hipStreamBeginCapture(gr->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(CSPD_E_DEVICE, "hipStreamBeginCapture failed");
        cspd_status rc;
        {
            ProfileSuspend quiet;
            if (p->s == 1)
                rc = cspd_omp_full(p, B, y, mask, k_fine, k_fine_uniform, support, coef, k_used, xhat, gr->capture);
            else
                rc = run_cross(p, B, y, mask, k_scale, k_fine, k_fine_uniform, support, coef, k_used, xhat,
                               support_coarse, (int32_t *)gr->work, c, gr->capture);
        }
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(gr->capture, &graph);
        gr->graph = graph;
        if (rc != CSPD_OK) {
            char msg[sizeof(cspd::g_err)];
            std::memcpy(msg, cspd::g_err, sizeof(msg));
            cspd_graph_destroy(gr);
            return set_error(rc, "%s", msg);
        }
        if (ce != hipSuccess || !graph) return fail(CSPD_E_DEVICE, "hipStreamEndCapture failed");
        if (hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0) != hipSuccess)
            return fail(CSPD_E_DEVICE, "hipGraphInstantiate failed");
        *out = gr;
        return CSPD_OK;
    });
}

cspd_status cspd_graph_launch(cspd_graph_t gr, void *hip_stream)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!gr || !gr->exec) return set_error(CSPD_E_INVALID, "graph is NULL");
        DeviceGuard g(gr->device);
        if (!g.ok) return set_error(CSPD_E_DEVICE, "hipSetDevice(%d) failed", gr->device);
        CSPD_HIP_CHECK(hipGraphLaunch(gr->exec, (hipStream_t)hip_stream));
        return CSPD_OK;
    });
}

void cspd_graph_destroy(cspd_graph_t gr)
{
    try {
        if (!gr) return;
        DeviceGuard g(gr->device);
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        if (gr->capture) {
            (void)hipStreamSynchronize(gr->capture);
            (void)hipStreamDestroy(gr->capture);
        }
        if (gr->work) {
            (void)hipDeviceSynchronize();   // no replay may still read the workspace
            (void)hipFree(gr->work);
        }
        delete gr;
    } catch (...) {
        // nothing may cross the C ABI; the object is left as it is
    }
}

cspd_status cspd_autotune(cspd_plan_t p, int64_t B, const void *y, const uint8_t *mask,
                          const int32_t *k_scale, const int32_t *k_fine, int32_t k_fine_uniform,
                          int32_t reps, void *hip_stream)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!p) return set_error(CSPD_E_INVALID, "plan is NULL");
        if (reps < 1 || reps > 1000) return set_error(CSPD_E_INVALID, "reps %d outside 1..1000", reps);
        if (p->s < 2 || p->dtype != CSPD_F32 || B == 0 || p->n_phases > 1) return CSPD_OK;   // nothing to choose
        CrossCall c;
        int32_t dummy = 0;
        cspd_status rc = prepare_cross(p, B, y, mask, k_scale, k_fine, k_fine_uniform, &dummy, &dummy, &dummy, c);
        if (rc != CSPD_OK) return rc;
        DeviceGuard g(p->device);
        if (!g.ok) return set_error(CSPD_E_DEVICE, "hipSetDevice(%d) failed", p->device);
        hipStream_t st = (hipStream_t)hip_stream;
        ProfileSuspend quiet;
        // scratch outputs and workspace for the timing runs
        int32_t *work = nullptr, *sup = nullptr, *ku = nullptr;
        void *coef = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto cleanup = [&]() {
            (void)hipStreamSynchronize(st);
            if (work) (void)hipFree(work);
            if (sup) (void)hipFree(sup);
            if (ku) (void)hipFree(ku);
            if (coef) (void)hipFree(coef);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        };
        const size_t wbytes = cross_workspace_bytes(p, B, c.ksum, false);
        if (hipMalloc((void **)&work, wbytes) != hipSuccess || hipMalloc((void **)&sup, sizeof(int32_t) * B * p->k_max) != hipSuccess ||
            hipMalloc((void **)&ku, sizeof(int32_t) * B) != hipSuccess ||
            hipMalloc(&coef, sizeof(float) * B * p->k_max) != hipSuccess) {
            cleanup();
            return set_error(CSPD_E_NOMEM, "autotune scratch for %lld patches", (long long)B);
        }
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            cleanup();
            return set_error(CSPD_E_DEVICE, "hipEventCreate failed");
        }
        // one call with the current choices leaves every coarse support in place
        rc = run_cross(p, B, y, mask, k_scale, k_fine, k_fine_uniform, sup, coef, ku, nullptr, nullptr, work, c, st);
        if (rc != CSPD_OK) { cleanup(); return rc; }
        const int64_t nk = B * (p->s - 1);
        for (int s = 0; s < p->s; ++s) {
            ScaleArgs a = cross_scale_args(p, s, B, y, mask, k_scale, k_fine, k_fine_uniform, sup, coef, ku, nullptr,
                                           work + nk, work, c.ksum);
            if (s == 0 && first_gemm_path(p)) {
                a.hpre = (char *)work + hpre_offset(p, B, c.ksum, false);
                a.nu2 = p->sc[0].nu2;
            }
            KernelChoice ch[24];
            const int nch = scale_choices(p->dtype, a, c.cand[s], p->sc[s].gram != nullptr, ch, 24);
            float best_ms = 0.f;
            int best = -1;
            for (int i = 0; i < nch; ++i) {
                if (launch_choice(p->dtype, a, ch[i], st) != CSPD_OK) { clear_error(); continue; }
                (void)hipEventRecord(e0, st);
                bool ok = true;
                for (int r = 0; r < reps && ok; ++r) ok = launch_choice(p->dtype, a, ch[i], st) == CSPD_OK;
                (void)hipEventRecord(e1, st);
                float ms = 0.f;
                if (!ok || hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    clear_error();
                    continue;
                }
                if (best < 0 || ms < best_ms) { best_ms = ms; best = i; }
            }
            if (best >= 0) {
                ch[best].cand = c.cand[s];
                std::lock_guard<std::mutex> lk(p->mu);
                p->tuned[s][k_bucket(a)] = ch[best];
            }
        }
        cleanup();
        return CSPD_OK;
    });
}

cspd_status cspd_tuned_kernel(cspd_plan_t p, int32_t scale, int32_t k_bucket_, int32_t *kind, int32_t *nc,
                              int32_t *ppw, int32_t *cand)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!p || !kind || !nc || !ppw || !cand) return set_error(CSPD_E_INVALID, "NULL argument");
        if (scale < 0 || scale >= p->s || k_bucket_ < 0 || k_bucket_ > 2)
            return set_error(CSPD_E_INVALID, "scale %d / bucket %d out of range", scale, k_bucket_);
        std::lock_guard<std::mutex> lk(p->mu);
        const KernelChoice &c = p->tuned[scale][k_bucket_];
        *kind = c.kind;
        *nc = c.nc;
        *ppw = c.ppw;
        *cand = c.cand;
        return CSPD_OK;
    });
}

cspd_status cspd_set_tuned_kernel(cspd_plan_t p, int32_t scale, int32_t k_bucket_, int32_t kind, int32_t nc,
                                  int32_t ppw, int32_t cand)
{
    return guarded([&]() -> cspd_status {
        clear_error();
        if (!p) return set_error(CSPD_E_INVALID, "plan is NULL");
        if (scale < 0 || scale >= p->s || k_bucket_ < 0 || k_bucket_ > 2)
            return set_error(CSPD_E_INVALID, "scale %d / bucket %d out of range", scale, k_bucket_);
        KernelChoice c;
        if (kind != kChoiceAuto) {
            if (cand < 1 || cand > p->sc[scale].t)
                return set_error(CSPD_E_INVALID, "cand %d outside [1, T = %d]", cand, p->sc[scale].t);
            // the variants that can run this scale at this candidate count
            ScaleArgs a = base_args(p, scale, 1, nullptr, nullptr);
            a.first = scale == 0;
            a.last = scale + 1 == p->s;
            a.kvec = nullptr;
            a.kuni = a.sup_count = 4 << k_bucket_;   // largest K of the bucket
            KernelChoice ch[24];
            const int nch = scale_choices(p->dtype, a, cand, p->sc[scale].gram != nullptr, ch, 24);
            int hit = -1;
            for (int i = 0; i < nch && hit < 0; ++i)
                if (ch[i].kind == kind && (kind == kChoiceFirstMfma || (ch[i].nc == nc && ch[i].ppw == ppw))) hit = i;
            if (hit < 0)
                return set_error(CSPD_E_UNSUPPORTED, "scale %d: no kernel kind %d (nc %d, ppw %d) for %d candidates",
                                 scale, kind, nc, ppw, cand);
            c = ch[hit];
            c.cand = cand;
        }
        std::lock_guard<std::mutex> lk(p->mu);
        p->tuned[scale][k_bucket_] = c;
        return CSPD_OK;
    });
}

}  // extern "C"
