"""HIP-graph capture of whole calls (MI355X only): every replay equals the
eager call bit for bit, with eager work and synchronisations between the
replays, and replays read the inputs as they are when they run."""
import numpy as np
import pytest

import gpu_util as G
import synth
from paper_1511_05174_amd import cspd

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


def test_graph_cross_scale_replays_match_eager():
    torch = G.torch_mod()
    w = synth.make("c2", batch=4096)
    plan = cspd.plan_from_workload(w)
    y, mask, kf, _ = G.inputs(w)
    ks = w.k_scales
    ref = [_np(t) for t in cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1])]
    g, sup, coef, ku, xh = cspd.cspd_graph_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1])
    for rep in range(4):
        sup.fill_(-9)
        xh.zero_()
        cspd.cspd_graph_launch(g)
        torch.cuda.synchronize()
        got = [_np(t) for t in (sup, coef, ku, xh)]
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), f"replay {rep}"
        # eager work between replays
        cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1])
        torch.cuda.synchronize()


def test_graph_reads_inputs_at_replay():
    torch = G.torch_mod()
    w1 = synth.make("c2", batch=2048)
    w2 = synth.make("c2", batch=2048, seed=99)
    plan = cspd.plan_from_workload(w1)
    y, mask, kf, _ = G.inputs(w1)
    y2, mask2, _, _ = G.inputs(w2)
    ks = w1.k_scales
    g, sup, coef, ku, xh = cspd.cspd_graph_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1])
    y.copy_(y2)
    mask.copy_(mask2)
    cspd.cspd_graph_launch(g)
    torch.cuda.synchronize()
    ref = cspd.cspd_omp_cross_scale(plan, y2, mask2, ks[:-1], kf, ks[-1])
    for a, b in zip(ref, (sup, coef, ku, xh)):
        assert np.array_equal(_np(a), _np(b))


def test_graph_single_scale_plan():
    torch = G.torch_mod()
    w = synth.custom([64], [256], batch=1000, seed=7, k_scales=[6], sigma=0.01, dtype="f32")
    plan = cspd.plan_from_workload(w)
    y, mask, kf, _ = G.inputs(w)
    ref = cspd.cspd_omp_full(plan, y, mask, kf, 6)
    g, sup, coef, ku, xh = cspd.cspd_graph_cross_scale(plan, y, mask, [], kf, 6)
    for _ in range(3):
        cspd.cspd_graph_launch(g)
        torch.cuda.synchronize()
        for a, b in zip(ref, (sup, coef, ku, xh)):
            assert np.array_equal(_np(a), _np(b))
