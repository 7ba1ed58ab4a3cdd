"""Time versus accuracy harness on the device (MI355X only): the video study
(single-scale full OMP over T atoms against zero-tree OMP, 8x8x32 patches)
and the Q study (cross-scale dictionaries trained per (T_low, Q)), at
reduced sizes.  The numbers themselves are measurements; the tests check
that the harness runs every point and that denoising behaves as the method
says it must on the model's signals."""
import numpy as np
import pytest

from paper_1511_05174_amd import timeacc

pytestmark = pytest.mark.gpu


def test_video_study_small():
    # 1024 patches: enough workgroups that neither path is bound by launch latency
    r = timeacc.video_time_accuracy(sizes=(256, 8192), ks=(8, 16), batch=1024, steps=2)
    z = r["zero_tree"]
    print(f"zero-tree: {z}", flush=True)
    for p in r["single_scale"]:
        print(p, flush=True)
    assert len(r["single_scale"]) == 4
    # every estimate denoises
    assert z["psnr_db"] > r["psnr_noisy_db"] + 3.0
    full = {(p["atoms"], p["k"]): p for p in r["single_scale"]}
    # the full fine dictionary represents the model's signals better than a
    # 256-atom piece of it, at the same sparsity
    assert full[(8192, 8)]["psnr_db"] > full[(256, 8)]["psnr_db"] + 1.0
    # zero-tree OMP searches 96 children instead of 8192 atoms
    assert z["ms_per_call"] < full[(8192, 8)]["ms_per_call"] / 2


def test_q_study_small():
    r = timeacc.q_effect(t_lows=(32,), qs=(2, 4), train_patches=2048, test_patches=512, iters_low=2,
                         iters_high=2, truth=(32, 4))
    print(r["points"], flush=True)
    assert len(r["points"]) == 2 and r["best_q"]["32"] in (2, 4)
    for p in r["points"]:
        assert np.isfinite(p["psnr_db"]) and p["psnr_db"] > 10.0
