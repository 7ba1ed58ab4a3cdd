"""Learning cross-scale dictionaries with the library (Section IV; MI355X
only): the sequence of zero-tree OMP and K-SVD updates runs, keeps unit
atoms, and lowers the representation error of the training set."""
import numpy as np
import pytest

import gpu_util as G
import synth
from paper_1511_05174_amd import cspd, train

pytestmark = pytest.mark.gpu


def test_cross_scale_learning_lowers_error():
    G.torch_mod()
    w = synth.make("c2", batch=4096)
    x = w.x.astype(np.float64)
    tm = {}
    d_low, d_high = train.cross_scale(x, w.up_maps[0], w.dims[0], w.atoms[0], w.atoms[1] // w.atoms[0],
                                      w.k_scales[0], w.k_scales[1], 2, 3, seed=1, timings=tm)
    assert d_low.shape == (w.atoms[0], w.dims[0]) and d_high.shape == (w.atoms[1], w.dims[1])
    assert np.all(np.isfinite(d_high)) and np.allclose(np.linalg.norm(d_high, axis=1), 1.0, atol=1e-5)
    assert len(tm["high"]) == 3 and len(tm["low"]) == 2
    # error of the learned pair vs the initial one (one zero-tree coding each)
    torch = G.torch_mod()
    X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()

    def err(dl, dh):
        plan = train._plan(list(w.dims), list(w.atoms), [dl.astype(np.float64), dh.astype(np.float64)],
                           [w.up_maps[0]], 8)
        sup, coef, _, xh = cspd.cspd_omp_cross_scale(plan, X, None, [w.k_scales[0]], None, w.k_scales[1])
        torch.cuda.synchronize()
        e = float(np.linalg.norm(xh.cpu().numpy() - x) / np.linalg.norm(x))
        cspd.cspd_plan_destroy(plan)
        return e

    rng = np.random.default_rng(1)
    xl = train.downsample(x, w.up_maps[0], w.dims[0])
    dl0 = train._unit_rows(xl[rng.choice(len(xl), size=w.atoms[0], replace=False)])
    dh0 = train._unit_rows(x[rng.choice(len(x), size=w.atoms[1], replace=False)])
    e0, e1 = err(dl0, dh0), err(d_low, d_high)
    print(f"[train] relative error initial {e0:.3f} learned {e1:.3f}", flush=True)
    assert e1 < e0
