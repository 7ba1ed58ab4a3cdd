"""Learning cross-scale dictionaries with the library (Section III-E; MI355X
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


def _unit(a):
    return a / np.linalg.norm(a, axis=1, keepdims=True)


def _coding_parity(w, sup, coef, full, ks):
    """Coding step against the oracle under the near-tie rule; returns the
    report (the caller bounds it)."""
    import parity
    gs = parity.gpu_scales(w, sup, np.count_nonzero(sup >= 0, axis=1).astype(np.int32),
                           None if full else None)
    return parity.compare(w, gs, coef.astype(np.float64), np.count_nonzero(sup >= 0, axis=1).astype(np.int32),
                          None, full=full, k_scales=ks, tie_tol=1e-6)


def _errors(x, d, sup, coef):
    """||x_j - sum_i coef_ji d_sup_ji|| in FP64 from the GPU's own supports and
    coefficients (the representation error the driver's heuristic reads)."""
    r = x.copy()
    for j in range(sup.shape[1]):
        m = sup[:, j] >= 0
        r[m] -= coef[m, j:j + 1].astype(np.float64) * d[sup[m, j]]
    return np.linalg.norm(r, axis=1)


def test_ksvd_iterations_match_the_oracle():
    """The training driver's plain K-SVD iteration (Algorithm 1 coding, the
    update sweep, heuristic 3) against the oracle, three iterations on the
    same dictionary: the coding by the near-tie rule, then the oracle's
    update sweep and heuristic 3 run on the GPU's supports and coefficients.
    Four initial atoms are exact copies of others: never picked (the lower
    index wins the tie), so heuristic 3 replaces them."""
    import dataclasses
    from oracle import ksvd as oks
    G.torch_mod()
    rng = np.random.default_rng(21)
    N, T, P, K = 16, 40, 800, 3
    dt = _unit(rng.standard_normal((T, N)))
    x = np.zeros((2 * P, N))
    for p in range(2 * P):
        a = rng.choice(T, size=K, replace=False)
        x[p] = rng.standard_normal(K) @ dt[a]
    x = (x + 0.01 * rng.standard_normal((2 * P, N))).astype(np.float32).astype(np.float64)
    # initial atoms from signals outside the training set (a training signal
    # that is itself an atom leaves a zero residual, where every pick ties)
    x, spare = x[:P], x[P:]
    d = _unit(spare[rng.choice(P, size=T - 4, replace=False)])
    d = np.vstack([d, d[:4]]).astype(np.float32)
    base = synth.custom([N], [T], P, seed=1, k_scales=[K], dtype="f32")
    torch = G.torch_mod()
    X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    D = torch.from_numpy(np.ascontiguousarray(d, dtype=np.float32)).cuda()
    total = 0
    for it in range(3):
        d = D.cpu().numpy()
        D, st = train.ksvd_step(X, x, D, K)
        dg, sg, cg, rg = D.cpu().numpy(), st["support"], st["coef"], [st["replaced"]]
        d64 = d.astype(np.float64)
        w = dataclasses.replace(base, dicts=[d64], x=x, y=x, mask=None, k_fine=None)
        rep = _coding_parity(w, sg, cg, True, [K])
        print(f"[ksvd it {it}] coding: {rep.summary()}; replaced {rg[0]}", flush=True)
        print("   excused/mismatched steps:", list(rep.detail.items())[:6], flush=True)
        rep.check(1e-5, 1e9, max_excused=P // 20)
        du, _, _ = oks.update(x, d64, sg, cg.astype(np.float64))
        err = _errors(x, d64, sg, cg)
        dn, repl = oks.replace_unused(du, x, sg, err)
        assert repl == rg[0]
        dev = float(np.max(np.abs(dg - dn)))
        print(f"[ksvd it {it}] largest atom difference {dev:.2e}", flush=True)
        assert dev < 1e-5
        total += len(repl)
    assert total >= 4


def test_cross_scale_iterations_match_the_oracle():
    """One step-2 iteration of the driver (zero-tree OMP coding, the update
    sweep, heuristic 4 with Omega_k from the coarse supports) against the
    oracle, three iterations: coding by the near-tie rule, update and
    heuristic 4 by the oracle on the GPU's supports, coefficients and coarse
    supports.  Some children start as copies of their siblings, so heuristic
    4 has atoms to replace."""
    import dataclasses
    from oracle import ksvd as oks
    torch = G.torch_mod()
    up, coarse = synth.box_map((4, 4), (2, 2))
    dims, atoms, kl, kh = [4, 16], [8, 32], 2, 3
    q = atoms[1] // atoms[0]
    w0 = synth.custom(dims, atoms, 600, seed=22, k_scales=[kl, kh], sigma=0.01, up_maps=[up], dict_kind="model",
                      dtype="f32")
    x = w0.y.astype(np.float32).astype(np.float64)      # the noisy signals
    d_low = w0.dicts[0].astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(23)
    dh = _unit(w0.dicts[1] + 0.05 * rng.standard_normal(w0.dicts[1].shape))
    dh[3] = dh[2]          # copies inside blocks 0 and 5: never picked
    dh[21] = dh[20]
    X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    D = torch.from_numpy(np.ascontiguousarray(dh, dtype=np.float32)).cuda()
    total = 0
    import parity
    for it in range(3):
        d64 = D.cpu().numpy().astype(np.float64)
        D, st = train.cross_scale_step(X, x, d_low, D, up, dims[0], q, kl, kh)
        w = dataclasses.replace(w0, dicts=[d_low, d64], x=x, y=x, mask=None, k_fine=None)
        ku = np.count_nonzero(st["support"] >= 0, axis=1).astype(np.int32)
        gs = parity.gpu_scales(w, st["support"], ku, st["coarse"], [kl])
        rep = parity.compare(w, gs, st["coef"].astype(np.float64), ku, None, k_scales=[kl, kh], tie_tol=1e-6)
        print(f"[cross it {it}] coding: {rep.summary()}; replaced {st['replaced']}", flush=True)
        print("   excused/mismatched steps:", list(rep.detail.items())[:6], flush=True)
        rep.check(1e-5, 1e9, max_excused=len(x) // 20)
        du, _, _ = oks.update(x, d64, st["support"], st["coef"].astype(np.float64))
        err = _errors(x, d64, st["support"], st["coef"])
        dn, repl = oks.replace_unused(du, x, st["support"], err, coarse_support=st["coarse"], q=q)
        assert repl == st["replaced"]
        dev = float(np.max(np.abs(D.cpu().numpy() - dn)))
        print(f"[cross it {it}] largest atom difference {dev:.2e}", flush=True)
        assert dev < 1e-5
        total += len(repl)
    assert total >= 2
