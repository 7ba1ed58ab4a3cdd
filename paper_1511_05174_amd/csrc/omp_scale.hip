// Kernel selection for one scale: patches per wavefront, candidate slots per
// lane and the register bucket for the sparsity, from the candidate count,
// the vector length and the requested sparsity.
#include "cspd_internal.h"

namespace cspd {

cspd_status dispatch_scale_f32_k4(const ScaleArgs &, int, int, int, bool, bool, hipStream_t);
cspd_status dispatch_scale_f32_k8(const ScaleArgs &, int, int, int, bool, bool, hipStream_t);
cspd_status dispatch_scale_f32_k16(const ScaleArgs &, int, int, int, bool, bool, hipStream_t);
cspd_status dispatch_scale_f64_k16(const ScaleArgs &, int, int, int, bool, hipStream_t);

namespace {

int pow2_at_least(int v)
{
    int p = 1;
    while (p < v) p *= 2;
    return p;
}

struct VecShape { int lp, nc, ppw; };
constexpr VecShape kVec[] = {{16, 1, 2}, {16, 2, 2}, {16, 4, 2}, {16, 4, 1}, {32, 1, 2}, {32, 2, 2},
                             {32, 2, 1}, {32, 4, 1}, {64, 1, 2}, {64, 1, 1}, {64, 2, 1}, {128, 1, 1}};

bool have_vec(int lp, int nc, int ppw)
{
    for (const VecShape &v : kVec)
        if (v.lp == lp && v.nc == nc && v.ppw == ppw) return true;
    return false;
}

}  // namespace

// Register-resident shape for `max_cand` candidates of length `lp`:
// two patches per wavefront when their vectors fit in 64 VGPRs, else one
// patch per wavefront within 128 VGPRs.  Returns false when neither fits.
bool scale_vec_shape(int lp, int max_cand, bool f64, int *nc, int *ppw)
{
    (void)f64;
    const int n2 = pow2_at_least((max_cand + 31) / 32);
    if (n2 * lp <= 64 && have_vec(lp, n2, 2)) { *nc = n2; *ppw = 2; return true; }
    const int n1 = pow2_at_least((max_cand + 63) / 64);
    if (n1 * lp <= 128 && have_vec(lp, n1, 1)) { *nc = n1; *ppw = 1; return true; }
    return false;
}

bool scale_vec_fits(int lp, int max_cand, bool f64)
{
    int nc, ppw;
    return scale_vec_shape(lp, max_cand, f64, &nc, &ppw);
}

// Whether the matrix-core Gram kernel has an instance for this shape.
bool mg_fits(int lp, int max_cand, int ppw)
{
    if (ppw == 2) return max_cand <= 32 && lp >= 16 && lp <= 128;
    return max_cand <= 64 && lp >= 32 && lp <= 128;
}

cspd_status dispatch_mg(const ScaleArgs &a, int ppw, int kreq, hipStream_t st)
{
    if (kreq <= 4) return dispatch_scale_f32_k4(a, a.lp, 1, ppw, false, true, st);
    if (kreq <= 8) return dispatch_scale_f32_k8(a, a.lp, 1, ppw, false, true, st);
    return dispatch_scale_f32_k16(a, a.lp, 1, ppw, false, true, st);
}

cspd_status launch_scale(int dtype, const ScaleArgs &a, int max_cand, bool gram, hipStream_t st)
{
    if (a.b <= 0) return CSPD_OK;
    int nc = 1, ppw = 1;
    if (gram) {
        nc = pow2_at_least((max_cand + 63) / 64);
        if (nc > 16 || a.lp > 256) return CSPD_E_UNSUPPORTED;
    } else if (!scale_vec_shape(a.lp, max_cand, dtype == CSPD_F64, &nc, &ppw)) {
        return CSPD_E_UNSUPPORTED;
    }
    const int k = a.sup_count < kMaxK ? a.sup_count : kMaxK;
    const int kreq = a.kvec ? k : (a.kuni < k ? a.kuni : k);
    if (dtype == CSPD_F64) return dispatch_scale_f64_k16(a, a.lp, nc, ppw, gram, st);
    // each patch's candidate Gram matrix on the matrix cores: up to 32
    // candidates with two patches per wavefront, up to 64 with one
    const bool mg = !gram && mg_fits(a.lp, max_cand, 2);
    if (mg) { nc = 1; ppw = 2; }
    else if (!gram && mg_fits(a.lp, max_cand, 1)) return dispatch_mg(a, 1, kreq, st);
    if (kreq <= 4) return dispatch_scale_f32_k4(a, a.lp, nc, ppw, gram, mg, st);
    if (kreq <= 8) return dispatch_scale_f32_k8(a, a.lp, nc, ppw, gram, mg, st);
    return dispatch_scale_f32_k16(a, a.lp, nc, ppw, gram, mg, st);
}

int k_bucket(const ScaleArgs &a)
{
    const int k = a.sup_count < kMaxK ? a.sup_count : kMaxK;
    const int kreq = a.kvec ? k : (a.kuni < k ? a.kuni : k);
    return kreq <= 4 ? 0 : (kreq <= 8 ? 1 : 2);
}

int scale_choices(int dtype, const ScaleArgs &a, int max_cand, bool has_gram, KernelChoice *out, int cap)
{
    int n = 0;
    auto add = [&](int kind, int nc, int ppw) {
        if (n < cap) { out[n].kind = kind; out[n].nc = nc; out[n].ppw = ppw; ++n; }
    };
    if (dtype != CSPD_F32) return 0;
    if (first_mfma_fits(dtype, a)) add(kChoiceFirstMfma, 1, 1);
    if (mg_fits(a.lp, max_cand, 2)) add(kChoiceMfmaGram, 1, 2);
    if (mg_fits(a.lp, max_cand, 1)) add(kChoiceMfmaGram, 1, 1);
    for (const VecShape &v : kVec)
        if (v.lp == a.lp && v.nc * (64 / v.ppw) >= max_cand) add(kChoiceVec, v.nc, v.ppw);
    if (has_gram) {
        const int nc = pow2_at_least((max_cand + 63) / 64);
        if (nc <= 16 && a.lp <= 256) add(kChoiceGram, nc, 1);
        if (nc <= 16 && proxy_gemm_fits(dtype, a)) add(kChoiceGemmGram, nc, 1);
    }
    return n;
}

cspd_status launch_choice(int dtype, const ScaleArgs &a, const KernelChoice &c, hipStream_t st)
{
    if (dtype != CSPD_F32) return CSPD_E_UNSUPPORTED;
    if (a.b <= 0) return CSPD_OK;
    ScaleArgs b = a;
    b.hpre = nullptr;   // only the GEMM variant has precomputed correlations
    if (c.kind == kChoiceGemmGram) {
        if (!a.hpre || !a.nu2) return CSPD_E_UNSUPPORTED;
        const cspd_status rc = launch_proxy_gemm(dtype, a, (float *)a.hpre, st);
        if (rc != CSPD_OK) return rc;
        b.hpre = a.hpre;
    }
    if (c.kind == kChoiceFirstMfma) return launch_first_mfma(dtype, b, st);
    const bool gram = c.kind == kChoiceGram || c.kind == kChoiceGemmGram, mg = c.kind == kChoiceMfmaGram;
    const int kb = k_bucket(b);
    if (kb == 0) return dispatch_scale_f32_k4(b, b.lp, c.nc, c.ppw, gram, mg, st);
    if (kb == 1) return dispatch_scale_f32_k8(b, b.lp, c.nc, c.ppw, gram, mg, st);
    return dispatch_scale_f32_k16(b, b.lp, c.nc, c.ppw, gram, mg, st);
}

}  // namespace cspd
