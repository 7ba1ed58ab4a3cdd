"""Structured measurement operators of the paper's experiments (Section IV)
against the FP64 oracle (MI355X only):

  * location-dependent coded exposure (videos): a per-pixel shutter tile
    whose shift depends on the patch position, i.e. one of 16 dense
    operators per patch (cspd_omp_cross_scale_phased);
  * Bayer demosaicing (images): 24x24 RGB patches seen through the
    colour-filter array at the patch's position, a per-patch mask over 1728
    samples (long-vector kernel at both scales);
  * coded-aperture light fields: two aperture codes over 4x4 views of 8x8
    pixels, one shared dense operator.
"""
import numpy as np
import pytest

import gpu_util as G
import oracle
import parity
import synth
from paper_1511_05174_amd import cspd
from test_gpu_parity import TOL, check_cross

pytestmark = pytest.mark.gpu


def run_phased(plan, w):
    torch = G.torch_mod()
    y, mask, kf, yh = G.inputs(w)
    ph = torch.from_numpy(np.ascontiguousarray(w.phase, dtype=np.int32)).cuda()
    ks = w.k_scales
    B = y.shape[0]
    sc = torch.full((B, int(sum(ks[:-1]))), -7, dtype=torch.int32, device=y.device)
    sup, coef, ku, xh = cspd.cspd_omp_cross_scale_phased(plan, ph, y, mask, ks[:-1], kf, ks[-1], support_coarse=sc)
    torch.cuda.synchronize()
    return dict(support=sup.cpu().numpy(), coef=coef.double().cpu().numpy(), k_used=ku.cpu().numpy(),
                xhat=xh.double().cpu().numpy(), support_coarse=sc.cpu().numpy(), y64=yh)


def test_coded_exposure_per_position():
    w = synth.make("c4loc", batch=1500)
    assert w.phi.shape == (16, 64, 512) and len(np.unique(w.phase)) == 16
    plan = cspd.plan_from_workload(w)
    out = run_phased(plan, w)
    ks = w.k_scales
    wo = G.with_y(w, out["y64"])
    sup = parity.gpu_scales(w, out["support"], out["k_used"], out["support_coarse"], ks[:-1])
    rep = parity.compare(wo, sup, out["coef"], out["k_used"], out["xhat"], k_scales=ks, tie_tol=TOL["f32"]["tie"])
    print(f"[coded exposure, 16 operators] {rep.summary()}", flush=True)
    rep.check(TOL["f32"]["coef"], TOL["f32"]["xhat"])
    # the operator matters: the same patches measured as if by operator 0
    # would not be what the oracle solved
    ref0 = oracle.omp_cross_scale(wo, phase=np.zeros(w.batch, dtype=np.int32))
    assert np.mean(np.all(ref0["support"] == out["support"][:, :ref0["support"].shape[1]], axis=1)) < 0.5


def test_phased_out_of_range_and_misuse():
    torch = G.torch_mod()
    w = synth.make("c4loc", batch=64)
    plan = cspd.plan_from_workload(w)
    ph = w.phase.copy()
    ph[[3, 10]] = [-1, 16]                      # outside [0, 16): not solved
    w2 = synth.subset(w, np.arange(w.batch))
    w2.phase = ph
    out = run_phased(plan, w2)
    assert out["k_used"][3] == 0 and out["k_used"][10] == 0
    assert np.all(out["support"][[3, 10]] == -1) and np.all(out["xhat"][[3, 10]] == 0)
    ok = np.setdiff1d(np.arange(w.batch), [3, 10])
    ref = run_phased(plan, synth.subset(w, ok))
    assert np.array_equal(out["support"][ok], ref["support"])
    # a plan with several operators only runs through the phased call
    y, mask, kf, _ = G.inputs(w)
    with pytest.raises(cspd.CspdError) as ei:
        cspd.cspd_omp_cross_scale(plan, y, mask, w.k_scales[:-1], kf, w.k_scales[-1])
    assert ei.value.code == cspd.E_INVALID
    with pytest.raises(cspd.CspdError):
        cspd.cspd_omp_cross_scale_phased(plan, None, y, mask, w.k_scales[:-1], kf, w.k_scales[-1])


def test_coded_exposure_grouping_skewed():
    """The first scale's correlations come from one GEMM over the batch
    grouped by operator: operators with no patch, one operator holding most
    of them (ragged last tile), a single-patch batch; against the oracle."""
    w = synth.make("c4loc", batch=700)
    rng = np.random.default_rng(12)
    ph = np.where(rng.random(w.batch) < 0.7, 3, rng.integers(4, 16, size=w.batch)).astype(np.int32)
    ph[ph == 5] = 6                             # operators 0, 1, 2 and 5 unused
    w2 = synth.subset(w, np.arange(w.batch))
    w2.phase = ph
    plan = cspd.plan_from_workload(w2)
    # (the measurements were taken with other operators: any y serves parity)
    for sub in (w2, synth.subset(w2, np.array([17]))):
        out = run_phased(plan, sub)
        ks = sub.k_scales
        wo = G.with_y(sub, out["y64"])
        sup = parity.gpu_scales(sub, out["support"], out["k_used"], out["support_coarse"], ks[:-1])
        rep = parity.compare(wo, sup, out["coef"], out["k_used"], out["xhat"], k_scales=ks,
                             tie_tol=TOL["f32"]["tie"])
        print(f"[coded exposure, skewed operators, B={sub.batch}] {rep.summary()}", flush=True)
        rep.check(TOL["f32"]["coef"], TOL["f32"]["xhat"])
    cspd.cspd_profile_reset()
    cspd.cspd_profile_enable(True)
    run_phased(plan, w2)
    cspd.cspd_profile_enable(False)
    assert "proxy_gemm<f32,groups>:s0" in cspd.cspd_profile_read()


def test_many_operators_grouping():
    """64 operators (four sign-flipped copies of the 16 coded-exposure
    shifts) over 900 patches: most operators hold a handful of patches, so
    almost every tile of the grouped first-scale GEMM is ragged; against the
    oracle."""
    import dataclasses
    w = synth.make("c4loc", batch=900)
    rng = np.random.default_rng(21)
    phis = np.concatenate([w.phi * rng.choice([-1.0, 1.0], size=(1, 1, w.phi.shape[2])) for _ in range(4)])
    ph = rng.integers(0, phis.shape[0], size=w.batch).astype(np.int32)
    w2 = dataclasses.replace(w, phi=phis, phase=ph)
    plan = cspd.plan_from_workload(w2)
    out = run_phased(plan, w2)
    ks = w2.k_scales
    wo = G.with_y(w2, out["y64"])
    sup = parity.gpu_scales(w2, out["support"], out["k_used"], out["support_coarse"], ks[:-1])
    rep = parity.compare(wo, sup, out["coef"], out["k_used"], out["xhat"], k_scales=ks, tie_tol=TOL["f32"]["tie"])
    print(f"[64 operators, B={w2.batch}] {rep.summary()}", flush=True)
    rep.check(TOL["f32"]["coef"], TOL["f32"]["xhat"])


def test_coded_exposure_full_size_sampled():
    """The bench's location-dependent coded-exposure batch (32,768 patches,
    16 operators: about 64 tiles per operator in the grouped GEMM); 256
    sampled patches against the oracle."""
    w = synth.make("c4loc")
    plan = cspd.plan_from_workload(w)
    out = run_phased(plan, w)
    idx = np.random.default_rng(4).choice(w.batch, 256, replace=False)
    ws = G.with_y(synth.subset(w, idx), out["y64"][idx])
    ks = w.k_scales
    sup = parity.gpu_scales(ws, out["support"][idx], out["k_used"][idx], out["support_coarse"][idx], ks[:-1])
    rep = parity.compare(ws, sup, out["coef"][idx], out["k_used"][idx], out["xhat"][idx], k_scales=ks,
                         tie_tol=TOL["f32"]["tie"])
    print(f"[coded exposure full-size sampled] {rep.summary()}", flush=True)
    rep.check(TOL["f32"]["coef"], TOL["f32"]["xhat"])


def test_bayer_demosaicing():
    w = synth.make("bayer", batch=300)
    # each patch observes one colour per pixel
    m = w.mask.reshape(-1, 24, 24, 3)
    assert np.all(m.sum(axis=3) == 1)
    check_cross(w)


def test_bayer_full_size_sampled():
    """The bench's Bayer batch (4,096 patches of 24x24x3 through the CFA:
    the long kernel's proxy loop and Gram mode in their launch
    configuration); 128 sampled patches against the oracle."""
    w = synth.make("bayer")
    plan = cspd.plan_from_workload(w)
    out = G.run_cross(plan, w)
    idx = np.random.default_rng(6).choice(w.batch, 128, replace=False)
    ws = G.with_y(synth.subset(w, idx), out["y64"][idx])
    ks = w.k_scales
    sup = parity.gpu_scales(ws, out["support"][idx], out["k_used"][idx], out["support_coarse"][idx], ks[:-1])
    rep = parity.compare(ws, sup, out["coef"][idx], out["k_used"][idx], out["xhat"][idx], k_scales=ks,
                         tie_tol=TOL["f32"]["tie"])
    print(f"[Bayer full-size sampled] {rep.summary()}", flush=True)
    rep.check(TOL["f32"]["coef"], TOL["f32"]["xhat"])


def test_coded_aperture_light_field():
    w = synth.make("lfca", batch=2000)
    assert w.phi.shape == (128, 1024)
    check_cross(w)
