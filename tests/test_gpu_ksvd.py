"""K-SVD dictionary update on the GPU against the FP64 oracle
(oracle/ksvd.py), and one cross-scale learning step (zero-tree OMP, then the
update) checked against the oracle update on the GPU's own supports
(MI355X only).  Tolerances: atoms and coefficients within 1e-4 (norm-wise,
per atom / per signal): FP32 data, FP64 Gram and power iteration."""
import numpy as np
import pytest

import gpu_util as G
import synth
from oracle import ksvd
from paper_1511_05174_amd import cspd

pytestmark = pytest.mark.gpu


def _problem(seed, P=3000, N=64, T=256, K=6, kstride=8):
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((T, N))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    sup = np.full((P, kstride), -1, dtype=np.int32)
    coef = np.zeros((P, kstride))
    for p in range(P):
        a = rng.choice(T - 3, size=K, replace=False)       # the last three atoms stay unused
        sup[p, :K] = a
        coef[p, :K] = rng.standard_normal(K)
    X = np.stack([coef[p, :K] @ D[sup[p, :K]] for p in range(P)]) + 0.3 * rng.standard_normal((P, N))
    D0 = D + 0.3 * rng.standard_normal((T, N))
    D0 /= np.linalg.norm(D0, axis=1, keepdims=True)
    return X.astype(np.float32), D0.astype(np.float32), sup, coef.astype(np.float32)


def _run_gpu(X, D, sup, coef):
    torch = G.torch_mod()
    x = torch.from_numpy(X).cuda()
    d = torch.from_numpy(D.copy()).cuda()
    s = torch.from_numpy(sup).cuda()
    c = torch.from_numpy(coef.copy()).cuda()
    cspd.cspd_ksvd_update(x, d, s, c)
    torch.cuda.synchronize()
    return d.cpu().numpy(), c.cpu().numpy()


def _check(X, D, sup, coef, dg, cg):
    Do, co, Ro = ksvd.update(X.astype(np.float64), D.astype(np.float64), sup, coef.astype(np.float64))
    datom = np.linalg.norm(dg - Do, axis=1)
    print(f"[ksvd] atom diff max {datom.max():.2e}", flush=True)
    assert datom.max() <= 1e-4
    used = sup >= 0
    cdiff = np.linalg.norm(np.where(used, cg - co, 0), axis=1) / np.maximum(np.linalg.norm(co, axis=1), 1e-30)
    print(f"[ksvd] coef diff max {cdiff.max():.2e}", flush=True)
    assert cdiff.max() <= 1e-4
    return Do, co, Ro


def test_update_matches_oracle():
    X, D, sup, coef = _problem(1)
    dg, cg = _run_gpu(X, D, sup, coef)
    _check(X, D, sup, coef, dg, cg)
    assert np.array_equal(dg[-3:], D[-3:])                   # unused atoms keep their value
    dg2, cg2 = _run_gpu(X, D, sup, coef)
    assert np.array_equal(dg, dg2) and np.array_equal(cg, cg2)   # deterministic


def test_update_small_atoms_and_heavy_users():
    """Coarse-scale atoms (N = 16) with many users each (several LDS chunks)."""
    X, D, sup, coef = _problem(2, P=4000, N=16, T=32, K=3, kstride=4)
    dg, cg = _run_gpu(X, D, sup, coef)
    _check(X, D, sup, coef, dg, cg)


def test_cross_scale_learning_step():
    """Step 2 of Section III-E on a small training set: zero-tree OMP with the
    current fine dictionary, then the update; the update is checked against
    the oracle on the GPU's own supports and coefficients."""
    torch = G.torch_mod()
    w = synth.make("c1", batch=1024)                       # identity operator, 8x8 / 4x4, FP64 data
    import dataclasses
    w = dataclasses.replace(w, dtype="f32")
    plan = cspd.plan_from_workload(w)
    y = torch.from_numpy(np.ascontiguousarray(w.y.astype(np.float32))).cuda()
    sup, coef, ku, xh = cspd.cspd_omp_cross_scale(plan, y, None, w.k_scales[:-1], None, w.k_scales[-1])
    torch.cuda.synchronize()
    X = w.y.astype(np.float32)
    D = w.dicts[-1].astype(np.float32).copy()              # (T, N): one atom per row
    S, Cf = sup.cpu().numpy(), coef.cpu().numpy()
    dg, cg = _run_gpu(X, D, S, Cf)
    Do, co, Ro = _check(X, D, S, Cf, dg, cg)
    before = np.linalg.norm(ksvd.residual(X.astype(np.float64), D.astype(np.float64), S, Cf.astype(np.float64)))
    assert np.linalg.norm(Ro) <= before + 1e-9
