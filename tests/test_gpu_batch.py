"""Full OMP in coefficient coordinates (Gram matrix precomputed, correlations
from one FP64 library GEMM) against the FP64 oracle (MI355X only): the
single-scale comparators of the paper's dictionary-size and time versus
accuracy studies (Section II-C, Section IV) -- up to 8192 atoms, vectors of
2048 coordinates (8x8x32 video patches), sparsity up to 64.  The batch is
small so that the oracle (Householder QR at every step) finishes in seconds.
"""
import numpy as np
import pytest

import gpu_util as G
import oracle
import parity
import synth
from paper_1511_05174_amd import cspd

pytestmark = pytest.mark.gpu

TIE, COEF, XHAT = 1e-6, 1e-5, 1e-5


def _labels(fn):
    cspd.cspd_profile_reset()
    cspd.cspd_profile_enable(True)
    out = fn()
    cspd.cspd_profile_enable(False)
    return out, sorted(cspd.cspd_profile_read())


def check_batch(w, k, k_max=16, max_excused=None):
    plan = cspd.plan_from_workload(w, k_max=k_max)
    out, labels = _labels(lambda: G.run_full(plan, w, k=k))
    assert any(l.startswith("omp_batch<") for l in labels), labels
    wo = G.with_y(w, out["y64"])
    sup = parity.gpu_scales(w, out["support"], out["k_used"])
    ks = list(w.k_scales)
    ks[-1] = k
    rep = parity.compare(wo, sup, out["coef"], out["k_used"], out["xhat"], full=True, k_scales=ks, tie_tol=TIE)
    print(f"[batch {w.name} T={w.atoms[-1]} L={w.m} K={k} B={w.batch}] {rep.summary()}", flush=True)
    rep.check(COEF, XHAT, max_excused=max_excused)
    cspd.cspd_plan_destroy(plan)
    return out, rep


def test_video_patches_2048_atoms():
    """8x8x32 video patches under the identity, 2048 atoms, K = 8."""
    w = synth.custom([2048], [2048], 48, seed=51, k_scales=[8], sigma=0.01, dtype="f32")
    check_batch(w, 8)


def test_8192_atoms():
    """The largest single-scale dictionary of the time versus accuracy study
    (8192 atoms), on 256-coordinate vectors, K = 12, a ragged batch."""
    w = synth.custom([256], [8192], 77, seed=52, k_scales=[12], sigma=0.01, dtype="f32")
    check_batch(w, 12)


def test_high_sparsity_dense_operator():
    """K = 40 through a shared Gaussian operator (512 measurements of 1024
    samples), 1024 atoms: the sparsity range of the dictionary-size study."""
    w = synth.custom([1024], [1024], 40, seed=53, phi_kind="dense", m=512, k_scales=[40], sigma=0.005,
                     dtype="f32")
    check_batch(w, 40, k_max=64)


def test_rank_and_dependent_atoms_stop():
    """24 measurements: no more than 24 atoms (the space is spanned); a
    duplicated atom never joins the support (it is dependent)."""
    w = synth.custom([256], [5000], 30, seed=54, phi_kind="dense", m=24, k_scales=[32], sigma=0.01,
                     dtype="f32")
    w.dicts[-1][1] = w.dicts[-1][0]
    # near the rank every remaining correlation is tiny: many steps are
    # near-ties, excused (and replayed) by the near-tie rule
    out, _ = check_batch(w, 32, k_max=32, max_excused=w.batch)
    assert np.all(out["k_used"] <= 24)
    for b in range(w.batch):
        s = set(out["support"][b, :out["k_used"][b]].tolist())
        assert not ({0, 1} <= s)


def test_per_patch_sparsity_and_zero():
    w = synth.custom([1024], [6000], 41, seed=55, k_scales=[10], sigma=0.01, dtype="f32")
    rng = np.random.default_rng(5)
    import dataclasses
    kf = rng.integers(0, 11, size=w.batch).astype(np.int32)
    kf[:3] = 0
    w = dataclasses.replace(w, k_fine=kf)
    out, _ = check_batch(w, 10)
    assert np.array_equal(out["k_used"][:3], [0, 0, 0])
