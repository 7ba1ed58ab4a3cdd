"""Kernel autotuner (MI355X only): every kernel variant that the tuner can
pick for a scale is checked against the FP64 oracle when pinned, and a tuned
plan gives oracle-exact supports with the fastest variant in place.  Same
tolerances as the other FP32 parity tests."""
import sys

import numpy as np
import pytest

import gpu_util as G
import parity
import synth
from paper_1511_05174_amd import cspd

pytestmark = pytest.mark.gpu

TIE, COEF, XHAT = 1e-6, 1e-5, 1e-5

# vector layouts (lp, nc, ppw) the library is built with, plus the other kinds
VEC = [(16, 1, 2), (16, 2, 2), (16, 4, 2), (16, 4, 1), (32, 1, 2), (32, 2, 2), (32, 2, 1), (32, 4, 1),
       (64, 1, 2), (64, 1, 1), (64, 2, 1), (128, 1, 1)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _bucket(k):
    return 0 if k <= 4 else (1 if k <= 8 else 2)


def _candidates(w, s):
    """Largest candidate count of scale s (all atoms at scale 0, else Q_s
    times the previous scale's sparsity, capped at T_s)."""
    if s == 0:
        return w.atoms[0]
    q = w.atoms[s] // w.atoms[s - 1]
    return min(q * w.k_scales[s - 1], w.atoms[s])


def _check(w, plan, label):
    out = G.run_cross(plan, w)
    ks = list(w.k_scales)
    wo = G.with_y(w, out["y64"])
    sup = parity.gpu_scales(w, out["support"], out["k_used"], out["support_coarse"], ks[:-1])
    rep = parity.compare(wo, sup, out["coef"], out["k_used"], out["xhat"], k_scales=ks, tie_tol=TIE)
    _say(f"[{label}] {rep.summary()}")
    rep.check(COEF, XHAT)
    return out


def _variants(plan, w, s):
    """Every (kind, nc, ppw) the library accepts for scale s of w."""
    cand = _candidates(w, s)
    b = _bucket(w.k_scales[s])
    found = []
    trials = [("first_mfma", 1, 1), ("mfma_gram", 1, 2), ("mfma_gram", 1, 1), ("gram", 1, 1), ("gram", 2, 1),
              ("gram", 4, 1), ("gemm_gram", 1, 1), ("gemm_gram", 2, 1), ("gemm_gram", 4, 1)]
    trials += [("vec", nc, ppw) for lp, nc, ppw in VEC]
    for kind, nc, ppw in trials:
        try:
            cspd.cspd_set_tuned_kernel(plan, s, b, kind, nc, ppw, cand)
        except cspd.CspdError:
            continue
        if (kind, nc, ppw) not in found:
            found.append((kind, nc, ppw))
    cspd.cspd_set_tuned_kernel(plan, s, b, "rules")
    return cand, b, found


@pytest.mark.parametrize("name,batch", [("c2", 1031), ("c4", 515), ("c3", 517), ("c5c", 263)])
def test_every_pinned_variant_matches_oracle(name, batch):
    w = synth.make(name, batch=batch)
    plan = cspd.plan_from_workload(w)
    for s in range(len(w.atoms)):
        cand, b, found = _variants(plan, w, s)
        assert found, f"scale {s}: no variant accepted"
        for kind, nc, ppw in found:
            cspd.cspd_set_tuned_kernel(plan, s, b, kind, nc, ppw, cand)
            assert cspd.cspd_tuned_kernel(plan, s, b)[0] == kind
            try:
                _check(w, plan, f"{name} scale {s} {kind} nc{nc} ppw{ppw}")
            except cspd.CspdError as e:
                # a variant may still be refused at launch (e.g. LDS limits)
                assert "cannot run this call" in str(e), str(e)
                _say(f"[{name} scale {s} {kind} nc{nc} ppw{ppw}] refused at launch: {e}")
        cspd.cspd_set_tuned_kernel(plan, s, b, "rules")


@pytest.mark.parametrize("name,batch", [("c2", 4093), ("c3", 1024)])
def test_autotuned_plan_matches_oracle(name, batch):
    w = synth.make(name, batch=batch)
    plan = cspd.plan_from_workload(w)
    y, mask, kf, _ = G.inputs(w)
    ks = w.k_scales
    cspd.cspd_autotune(plan, y, mask, ks[:-1], kf, ks[-1], reps=2)
    G.torch_mod().cuda.synchronize()
    for s in range(len(w.atoms)):
        kind, nc, ppw, cand = cspd.cspd_tuned_kernel(plan, s, _bucket(ks[s]))
        _say(f"[{name}] scale {s}: tuned {kind} nc{nc} ppw{ppw} cand{cand}")
        assert kind != "rules" and cand == _candidates(w, s)
    _check(w, plan, f"{name} autotuned")


def test_tuned_entry_keyed_by_candidate_count():
    """A pinned kernel is keyed by candidate count: with the coarse sparsity
    that gives that count the pinned kernel runs; a call whose coarse scale
    keeps fewer atoms (fewer candidates) falls back to the shape rules."""
    import dataclasses
    w = synth.make("c2", batch=1031)
    plan = cspd.plan_from_workload(w)
    s = 1
    cand = _candidates(w, s)                  # Q * K_low = 8 * 4 = 32
    b = _bucket(w.k_scales[s])
    cspd.cspd_set_tuned_kernel(plan, s, b, "vec", 1, 2, cand)
    cspd.cspd_profile_enable(True)
    try:
        for k_low, want in ((w.k_scales[0], "vec"), (w.k_scales[0] - 1, "mfma")):
            wk = dataclasses.replace(w, k_scales=[k_low, w.k_scales[1]])
            cspd.cspd_profile_reset()
            _check(wk, plan, f"c2 K_low {k_low}")
            labels = [lab for lab in cspd.cspd_profile_read() if lab.endswith(":s1")]
            _say(f"[c2 K_low {k_low}] scale-1 kernels {labels}")
            assert len(labels) == 1 and f"<f32,{want}," in labels[0], labels
    finally:
        cspd.cspd_profile_enable(False)


def test_set_tuned_kernel_rejects_bad_arguments():
    w = synth.make("c2", batch=16)
    plan = cspd.plan_from_workload(w)
    with pytest.raises(cspd.CspdError):
        cspd.cspd_set_tuned_kernel(plan, 5, 0, "vec", 1, 1, 4)
    with pytest.raises(cspd.CspdError):
        cspd.cspd_set_tuned_kernel(plan, 1, 3, "vec", 1, 1, 4)
    with pytest.raises(cspd.CspdError):
        cspd.cspd_set_tuned_kernel(plan, 1, 0, "vec", 1, 1, 0)
    with pytest.raises(cspd.CspdError):
        cspd.cspd_set_tuned_kernel(plan, 1, 0, "vec", 3, 5, 4)   # no such layout
    with pytest.raises(cspd.CspdError):
        cspd.cspd_autotune(plan, *G.inputs(w)[:2], w.k_scales[:-1], None, w.k_scales[-1], reps=0)
