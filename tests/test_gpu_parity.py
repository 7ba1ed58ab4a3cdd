"""HIP path against the FP64 oracle, through the C-ABI (MI355X only).

Tolerances: FP32 supports identical to the oracle's except near-ties whose
FP64 score gap is below 1e-6 of the largest step-1 score of that scale, at
most 1 + B/500 of them per run unless a test states its own bound; FP32
coefficients within 1e-5 of the patch's largest coefficient magnitude, entry
by entry; reconstructions within 1e-5 relative (norm-wise per patch); FP64
runs within 1e-10 with near-ties below 1e-9.
"""
import sys

import numpy as np
import pytest

import gpu_util as G
import parity
import synth
from paper_1511_05174_amd import cspd

pytestmark = pytest.mark.gpu

TOL = {"f32": dict(tie=1e-6, coef=1e-5, xhat=1e-5), "f64": dict(tie=1e-9, coef=1e-10, xhat=1e-10)}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_cross(w, dtype=None, k_scales=None, max_mismatch=0, max_excused=None):
    dtype = dtype or w.dtype
    plan = cspd.plan_from_workload(w, dtype=dtype)
    out = G.run_cross(plan, w, k_scales=k_scales, dtype=dtype)
    ks = list(k_scales if k_scales is not None else w.k_scales)
    wo = G.with_y(w, out["y64"])
    sup = parity.gpu_scales(w, out["support"], out["k_used"], out["support_coarse"], ks[:-1])
    rep = parity.compare(wo, sup, out["coef"], out["k_used"], out["xhat"], k_scales=ks,
                         tie_tol=TOL[dtype]["tie"])
    _say(f"[cross {w.name} B={w.batch} {dtype}] {rep.summary()}")
    rep.check(TOL[dtype]["coef"], TOL[dtype]["xhat"], max_excused=max_excused, max_mismatch=max_mismatch)
    return out, rep


def check_full(w, dtype=None, k=None, max_excused=None):
    dtype = dtype or w.dtype
    plan = cspd.plan_from_workload(w, dtype=dtype)
    out = G.run_full(plan, w, k=k, dtype=dtype)
    wo = G.with_y(w, out["y64"])
    sup = parity.gpu_scales(w, out["support"], out["k_used"])
    ks = list(w.k_scales)
    if k is not None:
        ks[-1] = k
    rep = parity.compare(wo, sup, out["coef"], out["k_used"], out["xhat"], full=True, k_scales=ks,
                         tie_tol=TOL[dtype]["tie"])
    _say(f"[full {w.name} B={w.batch} {dtype}] {rep.summary()}")
    rep.check(TOL[dtype]["coef"], TOL[dtype]["xhat"], max_excused=max_excused)
    return out, rep


# ---------------------------------------------------------------- workloads
def test_c1_fp64_cross():
    check_cross(synth.make("c1"))


def test_c1_fp64_full():
    check_full(synth.make("c1"))


def test_c1_indep_dicts_fp32():
    check_cross(synth.make("c1", batch=2048, dict_kind="indep"), dtype="f32")


def test_c2_cross_ragged():
    check_cross(synth.make("c2", batch=4093))


def test_c3_cross():
    check_cross(synth.make("c3", batch=2048))


def test_c4_cross_uneven_k():
    out, _ = check_cross(synth.make("c4", batch=2051))
    assert out["k_used"].min() >= 4


@pytest.mark.parametrize("name", ["c5a", "c5b", "c5c"])
def test_c5_shapes_cross(name):
    check_cross(synth.make(name, batch=1031))


# --------------------------------------------------------------- edge cases
def test_empty_batch():
    w = synth.make("c2", batch=4)
    plan = cspd.plan_from_workload(w)
    torch = G.torch_mod()
    y = torch.zeros((0, 64), dtype=torch.float32, device="cuda")
    m = torch.zeros((0, 64), dtype=torch.uint8, device="cuda")
    sup, coef, ku, xh = cspd.cspd_omp_cross_scale(plan, y, m, [4], None, 8)
    assert sup.shape == (0, plan.k_max)


@pytest.mark.parametrize("b", [1, 3, 5, 65])
def test_tiny_batches(b):
    check_cross(synth.make("c2", batch=b))


def test_zero_and_capped_sparsity():
    w = synth.make("c4", batch=300)
    kf = w.k_fine.copy()
    kf[::7] = 0
    import dataclasses
    w = dataclasses.replace(w, k_fine=kf)
    out, _ = check_cross(w)
    assert np.all(out["k_used"][::7] == 0)
    assert np.all(out["support"][::7] == -1)
    # K above Q * K_low is capped at the candidate count
    w2 = synth.custom([16, 64], [32, 64], batch=257, seed=5, k_scales=[2, 16], sigma=0.05,
                      dict_kind="model", dtype="f32")
    out2, _ = check_cross(w2)
    assert out2["k_used"].max() <= 4


def test_unobserved_patch():
    w = synth.make("c2", batch=130)
    w.mask[5] = 0
    w.y[5] = 0
    w.mask[6, 1:] = 0
    out, _ = check_cross(w)
    assert out["k_used"][5] == 0
    assert out["k_used"][6] <= 1


def test_dependent_atoms_stop():
    """Duplicated atoms: the copy is never merged (it is dependent)."""
    w = synth.custom([8, 16], [4, 16], batch=129, seed=9, k_scales=[2, 8], sigma=0.1, dtype="f32")
    w.dicts[1][1] = w.dicts[1][0]
    w.dicts[1][5] = -w.dicts[1][4]
    # a duplicate ties its original exactly (gap 0) whenever either is the best
    # remaining atom, so these patches are allowed more excusals
    out, _ = check_cross(w, max_excused=12)
    for b in range(w.batch):
        s = set(out["support"][b, :out["k_used"][b]])
        assert not ({0, 1} <= s) and not ({4, 5} <= s)


def test_single_parent_equals_full():
    """T_0 = 1: zero-tree OMP searches every fine atom, like Algorithm 1."""
    w = synth.custom([4, 32], [1, 96], batch=300, seed=3, k_scales=[1, 6], sigma=0.05, dtype="f32")
    a, _ = check_cross(w)
    b, _ = check_full(w, k=6)
    assert np.array_equal(a["support"], b["support"])


def test_three_scale_fp64():
    w = synth.custom([4, 16, 64], [8, 32, 128], batch=513, seed=4, k_scales=[2, 4, 6], sigma=0.02,
                     phi_kind="dense", m=48, dict_kind="model", dtype="f64")
    check_cross(w)


def test_full_gram_path():
    w = synth.custom([16, 64], [64, 512], batch=700, seed=6, k_scales=[4, 8], sigma=0.01,
                     phi_kind="dense", m=40, dict_kind="model", dtype="f32")
    check_full(w)


def test_dense_first_scale_gemm_ragged():
    """Scale 0 under a shared dense operator runs the batched correlation GEMM
    and the Gram-table kernel: atoms not a multiple of the 32-atom block,
    a measurement length not a multiple of 4 and a ragged last wavefront."""
    w = synth.custom([16, 64], [48, 384], batch=1003, seed=12, k_scales=[3, 6], sigma=0.01,
                     phi_kind="dense", m=36, dict_kind="model", dtype="f32")
    cspd.cspd_profile_reset()
    cspd.cspd_profile_enable(True)
    try:
        check_cross(w)
        labels = list(cspd.cspd_profile_read())
    finally:
        cspd.cspd_profile_enable(False)
    assert any(lab.startswith("proxy_gemm") for lab in labels), labels
    assert any("gram" in lab and lab.endswith(":s0") for lab in labels), labels


def test_one_patch_mfma_gram_partial_blocks():
    """Up to 64 candidates on one patch per wavefront, vectors of 32
    coordinates (16 per lane half, a single chunk)."""
    w = synth.custom([16, 64], [32, 512], batch=777, seed=13, k_scales=[4, 10], sigma=0.02,
                     phi_kind="dense", m=32, dict_kind="model", dtype="f32")
    cspd.cspd_profile_reset()
    cspd.cspd_profile_enable(True)
    try:
        check_cross(w)
        labels = list(cspd.cspd_profile_read())
    finally:
        cspd.cspd_profile_enable(False)
    assert any("mfma" in lab and "ppw1" in lab and lab.endswith(":s1") for lab in labels), labels


@pytest.mark.parametrize("alpha", [1e-5, 1e5])
def test_split_gram_dictionary_scale(alpha):
    # the two-patch matrix-core Gram works on FP16 parts of the weighted
    # candidates scaled by a power of two chosen at plan time: dictionaries
    # far from unit norm (and measurements of their size) keep the FP32 bar
    import dataclasses
    w = synth.make("c2", batch=2048)
    ws = dataclasses.replace(w, dicts=[d * alpha for d in w.dicts], y=w.y * alpha, x=w.x * alpha)
    check_cross(ws)


def test_three_scale_mask_blocks_split_gram():
    # a masked 3-scale plan whose middle scale folds blocks of four fine
    # samples (weights sqrt(observed) up to 2): the split Gram's scale covers
    # the weights, and the middle scale runs the two-patch matrix-core Gram
    import dataclasses
    from synth.workloads import box_map
    w = synth.make("c2", batch=4096)
    rng = np.random.default_rng(11)
    d0 = rng.standard_normal((32, 4))
    d0 /= np.linalg.norm(d0, axis=1, keepdims=True)
    up01 = box_map((4, 4), (2, 2))[0].astype(np.int32)
    w3 = dataclasses.replace(w, dims=[4, 16, 64], atoms=[32, 128, 1024], dicts=[d0, w.dicts[0], w.dicts[1]],
                             up_maps=[up01, w.up_maps[0]], k_scales=[2, 4, 8])
    check_cross(w3)


def test_children_not_a_power_of_two():
    # q = 3 children per coarse atom: the child map's division by q is a
    # high multiply by a plan-time reciprocal
    import dataclasses
    w = synth.make("c1", batch=2048)
    w3 = dataclasses.replace(w, atoms=[64, 192], dicts=[w.dicts[0], w.dicts[1][:192]])
    check_cross(w3, dtype="f32")


def test_deterministic():
    w = synth.make("c3", batch=1500)
    plan = cspd.plan_from_workload(w)
    a = G.run_cross(plan, w)
    b = G.run_cross(plan, w)
    for k in ("support", "coef", "k_used", "xhat"):
        assert np.array_equal(a[k], b[k]), k


def test_batch_invariance():
    """A patch's result does not depend on the other patches of the launch."""
    w = synth.make("c2", batch=3000)
    plan = cspd.plan_from_workload(w)
    a = G.run_cross(plan, w)
    idx = np.arange(100, 1700, 7)
    b = G.run_cross(plan, synth.subset(w, idx))
    for k in ("support", "coef", "k_used", "xhat"):
        assert np.array_equal(a[k][idx], b[k]), k


# ------------------------------------------------- full-size sampled parity
def test_c2_full_size_sampled():
    """The 65,536-patch inpainting workload in the benchmark's configuration;
    256 sampled patches checked against the oracle."""
    w = synth.make("c2")
    plan = cspd.plan_from_workload(w)
    out = G.run_cross(plan, w)
    idx = np.random.default_rng(0).choice(w.batch, 256, replace=False)
    ws = G.with_y(synth.subset(w, idx), out["y64"][idx])
    ks = w.k_scales
    sup = parity.gpu_scales(ws, out["support"][idx], out["k_used"][idx], out["support_coarse"][idx], ks[:-1])
    rep = parity.compare(ws, sup, out["coef"][idx], out["k_used"][idx], out["xhat"][idx], tie_tol=1e-6)
    _say(f"[cross c2 full-size sampled] {rep.summary()}")
    rep.check(1e-5, 1e-5)


# ------------------------------------------- full OMP on matrix cores (large T)
def test_c2_full_mfma_masked():
    check_full(synth.make("c2", batch=2053))


def test_c3_full_mfma_dense():
    check_full(synth.make("c3", batch=1024))


def test_c4_full_mfma_uneven_k():
    out, _ = check_full(synth.make("c4", batch=1029))
    assert out["k_used"].min() >= 4


def test_c5c_full_mfma_lightfield():
    check_full(synth.make("c5c", batch=515))


# ------------------------------------ first scale on the matrix cores (GEMM)
@pytest.mark.parametrize("t0,k_low", [(32, 3), (64, 8), (128, 5)])
def test_first_scale_mask_shapes(t0, k_low):
    """Coarse dictionaries of one, two and four 32-atom tiles, sparsity up to 8."""
    w = synth.custom([16, 64], [t0, t0 * 4], batch=1029, seed=11 + t0, phi_kind="mask",
                     k_scales=[k_low, 6], sigma=0.005, dict_kind="model", dtype="f32")
    check_cross(w)


def test_first_scale_dense_operator():
    """Shared Gaussian operator of 24 rows: the coarse candidates are the
    columns of Phi U D_0 (length 24), on the matrix-core first scale."""
    w = synth.custom([16, 64], [64, 256], batch=777, seed=21, phi_kind="dense", m=24,
                     k_scales=[4, 6], sigma=0.005, dict_kind="model", dtype="f32")
    check_cross(w)


def test_first_scale_duplicate_atoms():
    """Duplicated and negated coarse atoms: exact ties go to the lower index
    and the copy never joins the support (it is dependent)."""
    w = synth.custom([16, 64], [32, 128], batch=515, seed=23, phi_kind="mask",
                     k_scales=[6, 6], sigma=0.005, dict_kind="model", dtype="f32")
    d0 = w.dicts[0]
    d0[1] = d0[0]
    d0[5] = -d0[4]
    out, _ = check_cross(w)
    for b in range(w.batch):
        s = set(out["support_coarse"][b, :6].tolist())
        assert not ({0, 1} <= s) and not ({4, 5} <= s)


