"""Pins for the FP64 oracle: checks against facts the paper and the mathematics
fix, independent of the oracle's own arithmetic.

Each ``pin_*`` function raises AssertionError when the oracle compiled at
``lib`` disagrees.  The same functions run against the real oracle
(test_oracle_pins.py) and against deliberately broken copies of it
(test_oracle_mutants.py), where at least one pin must fire.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import scipy.linalg

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "omp_tiny.json")


def _single(dict_atoms, y, k, lib, phi_kind="identity", phi=None, mask=None, **kw):
    d = np.asarray(dict_atoms, dtype=np.float64)
    t, n = d.shape
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    m = y.shape[1]
    return oracle.omp([n], [t], [d], [], phi_kind, m, phi, y, mask, [k], lib_path=lib, **kw)


def _lstsq_residual(a, y):
    beta, *_ = np.linalg.lstsq(a, y, rcond=None)
    return y - a @ beta, beta


# --------------------------------------------------------------------------
# Golden fixtures worked by hand from Algorithm 1 / Algorithm 2.
# --------------------------------------------------------------------------
def pin_golden(lib):
    g = json.load(open(GOLDEN))
    for case in g["cases"]:
        out = _single(case["dict_atoms"], case["y"], case["k"][0], lib)
        ku = int(out["k_used"][0, 0])
        assert ku == case["k_used"], (case["name"], ku)
        assert list(out["support"][0, :ku]) == case["support"], (case["name"], out["support"][0])
        np.testing.assert_allclose(out["coef"][0, :ku], case["coef"], rtol=1e-12, atol=1e-12)
    for case in g["cross_scale_cases"]:
        dicts = [np.asarray(a, dtype=np.float64) for a in case["dict_atoms"]]
        ups = [np.asarray(u, dtype=np.int32) for u in case["up_maps"]]
        y = np.asarray([case["y"]], dtype=np.float64)
        cs = oracle.omp(case["dims"], case["atoms"], dicts, ups, "identity", case["dims"][-1], None,
                        y, None, case["k"], lib_path=lib)
        assert list(cs["support"][0, :case["k_used"]]) == case["support"], cs["support"]
        np.testing.assert_allclose(cs["coef"][0, :case["k_used"]], case["coef"], rtol=1e-12, atol=1e-12)
        fu = oracle.omp(case["dims"], case["atoms"], dicts, ups, "identity", case["dims"][-1], None,
                        y, None, case["k"], full=True, lib_path=lib)
        assert list(fu["support"][0, :2]) == case["full_support"], fu["support"]
        np.testing.assert_allclose(fu["coef"][0, :2], case["full_coef"], rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# P1: brute force on tiny inputs.
# --------------------------------------------------------------------------
def pin_bruteforce_greedy(lib, trials=40, seed=11):
    """Each greedy step picks the candidate with the largest |<a_i, r>|/||a_i||,
    where r is recomputed with LAPACK least squares on the oracle's own prefix;
    the final coefficients are the least-squares optimum on the final support;
    and the exhaustive l0 optimum over all K-subsets never exceeds OMP's
    residual."""
    rng = np.random.default_rng(seed)
    for _ in range(trials):
        m, t, k = int(rng.integers(4, 8)), int(rng.integers(6, 12)), int(rng.integers(1, 4))
        d = rng.standard_normal((t, m))
        d[rng.integers(0, t)] *= 3.0          # non-unit atom: normalisation matters
        y = rng.standard_normal(m)
        out = _single(d, y, k, lib)
        ku = int(out["k_used"][0, 0])
        sup = list(out["support"][0, :ku])
        assert ku == k
        a = d.T
        nu = np.linalg.norm(a, axis=0)
        for n in range(ku):
            prefix = sup[:n]
            r = y.copy() if n == 0 else _lstsq_residual(a[:, prefix], y)[0]
            scores = np.abs(a.T @ r) / nu
            scores[prefix] = -1
            assert scores[sup[n]] >= scores.max() - 1e-12, (n, sup, scores)
        res, beta = _lstsq_residual(a[:, sup], y)
        np.testing.assert_allclose(out["coef"][0, :ku], beta, rtol=1e-9, atol=1e-12)
        best = min(np.linalg.norm(_lstsq_residual(a[:, list(c)], y)[0])
                   for c in itertools.combinations(range(t), k))
        assert np.linalg.norm(res) >= best - 1e-12


def pin_bruteforce_cross_scale(lib, trials=25, seed=12):
    """Cross-scale: every fine atom lies in a child block of a coarse pick, the
    coarse picks are greedy-optimal for (P_low), the fine picks are greedy over
    the children only, and the fine coefficients are the least-squares
    optimum on the fine support."""
    rng = np.random.default_rng(seed)
    for _ in range(trials):
        n_c, n_f, t0, q = 2, 4, 4, 2
        k0, k1 = 2, 2
        up = np.array([0, 0, 1, 1], dtype=np.int32)
        d0 = rng.standard_normal((t0, n_c))
        d1 = rng.standard_normal((t0 * q, n_f))
        y = rng.standard_normal(n_f)
        out = oracle.omp([n_c, n_f], [t0, t0 * q], [d0, d1], [up], "identity", n_f, None, y[None],
                         None, [k0, k1], lib_path=lib)
        coarse = list(out["supports"][0, 0, :out["k_used"][0, 0]])
        fine = list(out["supports"][0, 1, :out["k_used"][0, 1]])
        # (P_low) greedy check in measurement space: effective atoms U d
        a0 = d0[:, up].T
        nu0 = np.linalg.norm(a0, axis=0)
        for n, pick in enumerate(coarse):
            r = y if n == 0 else _lstsq_residual(a0[:, coarse[:n]], y)[0]
            sc = np.abs(a0.T @ r) / nu0
            sc[coarse[:n]] = -1
            assert sc[pick] >= sc.max() - 1e-12
        for f in fine:
            assert f // q in coarse, (fine, coarse)
        a1 = d1.T
        cand = sorted(c * q + j for c in coarse for j in range(q))
        nu1 = np.linalg.norm(a1, axis=0)
        for n, pick in enumerate(fine):
            r = y if n == 0 else _lstsq_residual(a1[:, fine[:n]], y)[0]
            sc = np.full(t0 * q, -1.0)
            sc[cand] = np.abs(a1[:, cand].T @ r) / nu1[cand]
            sc[fine[:n]] = -1
            assert sc[pick] >= sc.max() - 1e-12
        res, beta = _lstsq_residual(a1[:, fine], y)
        np.testing.assert_allclose(out["coef"][0, :len(fine)], beta, rtol=1e-9, atol=1e-12)


# --------------------------------------------------------------------------
# P2: exact recovery (mutual coherence guarantee).
# --------------------------------------------------------------------------
def dirac_hadamard(n=64):
    h = scipy.linalg.hadamard(n) / np.sqrt(n)
    return np.vstack([np.eye(n), h.T])  # (2n, n) atoms


def pin_exact_recovery(lib, trials=200, seed=13):
    """Dirac + Hadamard (64 x 128) has coherence 1/8; every noiseless s-sparse
    signal with s < (1 + 8)/2 is recovered exactly by OMP (Tropp 2004,
    Donoho & Elad 2003), support and coefficients."""
    d = dirac_hadamard(64)
    rng = np.random.default_rng(seed)
    b = trials
    ys, sups, cfs = [], [], []
    for _ in range(b):
        s = int(rng.integers(1, 5))
        sup = rng.choice(128, size=s, replace=False)
        cf = rng.standard_normal(s) + np.sign(rng.standard_normal(s)) * 0.5
        ys.append(d[sup].T @ cf)
        sups.append(sup)
        cfs.append(cf)
    for i in range(b):
        out = _single(d, ys[i], len(sups[i]), lib)
        ku = int(out["k_used"][0, 0])
        assert ku == len(sups[i])
        got = out["support"][0, :ku]
        assert set(got) == set(sups[i]), (got, sups[i])
        order = [list(got).index(j) for j in sups[i]]
        np.testing.assert_allclose(out["coef"][0, order], cfs[i], rtol=1e-10, atol=1e-12)


def pin_exact_recovery_cross_scale(lib, trials=100, seed=14):
    """Model-consistent two-scale data: children of a coarse atom are its
    upsampled copy plus detail the box average removes, so W x is exactly
    sparse on the parents.  With a coarse Dirac + Hadamard dictionary (16 x 32,
    coherence 1/4) and at most 2 active parents, noiseless (P_low) recovers the
    parents, and the fine step, restricted to their children, recovers the
    signal with zero residual."""
    rng = np.random.default_rng(seed)
    n_c, n_f, q = 16, 64, 4
    d0 = dirac_hadamard(16)                       # (32, 16)
    up = (np.arange(64).reshape(8, 8)[::1, ::1] * 0).reshape(-1)
    ii, jj = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    up = ((ii // 2) * 4 + (jj // 2)).reshape(-1).astype(np.int32)
    d1 = np.zeros((32 * q, 64))
    for p in range(32):
        base = d0[p][up]
        for c in range(q):
            g = rng.standard_normal(64)
            gm = np.zeros(16)
            np.add.at(gm, up, g)
            g = g - (gm / 4)[up]
            v = base / 2.0 + 0.3 * g / 8.0
            d1[p * q + c] = v / np.linalg.norm(v)
    for _ in range(trials):
        parents = rng.choice(32, size=2, replace=False)
        kids = np.array([parents[0] * q + rng.integers(q), parents[1] * q + rng.integers(q)])
        cf = rng.standard_normal(2) + np.sign(rng.standard_normal(2))
        # keep both parents visible at the coarse scale
        x = d1[kids].T @ cf
        out = oracle.omp([n_c, n_f], [32, 32 * q], [d0, d1], [up], "identity", n_f, None, x[None],
                         None, [2, 2], lib_path=lib)
        coarse = set(out["supports"][0, 0, :2])
        wx = np.zeros(16)
        np.add.at(wx, up, x)
        wx /= 4
        # coarse truth: W x = sum_c cf_c * (W d_kid_c), each W d_kid ∝ d0[parent]
        assert coarse == set(parents), (coarse, parents)
        xh = out["xhat"][0]
        assert np.linalg.norm(x - xh) <= 1e-9 * np.linalg.norm(x)


# --------------------------------------------------------------------------
# P3: orthonormal dictionary -> sorting Dᵀy.
# --------------------------------------------------------------------------
def pin_orthonormal(lib, trials=30, seed=15):
    rng = np.random.default_rng(seed)
    for _ in range(trials):
        n = int(rng.integers(4, 20))
        qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
        d = qm.T                                  # atoms = orthonormal columns
        y = rng.standard_normal(n)
        k = int(rng.integers(1, n))
        out = _single(d, y, k, lib)
        c = qm.T @ y
        want = np.argsort(-np.abs(c), kind="stable")[:k]
        assert list(out["support"][0, :k]) == list(want)
        np.testing.assert_allclose(out["coef"][0, :k], c[want], rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------
# P4: invariants.
# --------------------------------------------------------------------------
def pin_invariants(lib, seed=16):
    """Residual orthogonal to the selected atoms; ||r||^2 = ||y||^2 - ||P y||^2;
    residual norm non-increasing in K; the K-1 run is a prefix of the K run;
    supports are distinct and inside the candidate set."""
    import synth
    w = synth.custom([16, 64], [64, 256], batch=64, seed=seed, k_scales=[3, 6], sigma=0.05,
                     phi_kind="dense", m=40)
    a = w.phi @ w.dicts[1].T                       # effective fine dictionary, (M, T)
    prev_res = None
    prev_sup = None
    for k in range(1, 7):
        out = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, w.phi_kind, w.m, w.phi, w.y, None,
                         [3, k], full=True, lib_path=lib)
        res_norms = []
        for b in range(w.batch):
            ku = int(out["k_used"][b, 1])
            sup = out["support"][b, :ku]
            assert len(set(sup)) == ku and ku == k
            r = w.y[b] - a[:, sup] @ out["coef"][b, :ku]
            assert np.linalg.norm(a[:, sup].T @ r) <= 1e-10 * np.linalg.norm(a) * np.linalg.norm(w.y[b])
            q, _ = np.linalg.qr(a[:, sup])
            py = q @ (q.T @ w.y[b])
            assert abs(r @ r - (w.y[b] @ w.y[b] - py @ py)) <= 1e-10 * (w.y[b] @ w.y[b])
            res_norms.append(np.linalg.norm(r))
            if prev_sup is not None:
                assert list(prev_sup[b]) == list(sup[:k - 1])
        res_norms = np.array(res_norms)
        if prev_res is not None:
            assert np.all(res_norms <= prev_res + 1e-12)
        prev_res = res_norms
        prev_sup = out["support"][:, :k].copy()


# --------------------------------------------------------------------------
# P5: reductions to full OMP.
# --------------------------------------------------------------------------
def pin_reductions(lib, seed=17):
    """One coarse atom owning every fine atom (T_0 = 1), or selecting every
    coarse atom (K_0 = T_0 <= M), leaves the fine search over all atoms, so
    zero-tree OMP must equal Algorithm 1 exactly."""
    import synth
    w = synth.custom([4, 32], [1, 96], batch=48, seed=seed, k_scales=[1, 5], sigma=0.1)
    cs = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "identity", w.m, None, w.y, None, [1, 5], lib_path=lib)
    fu = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "identity", w.m, None, w.y, None, [1, 5], full=True, lib_path=lib)
    assert np.array_equal(cs["support"], fu["support"])
    assert np.array_equal(cs["coef"], fu["coef"])
    w = synth.custom([8, 32], [6, 48], batch=48, seed=seed + 1, k_scales=[6, 5], sigma=0.1)
    cs = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "identity", w.m, None, w.y, None, [6, 5], lib_path=lib)
    fu = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "identity", w.m, None, w.y, None, [6, 5], full=True, lib_path=lib)
    assert np.all(cs["k_used"][:, 0] == 6)
    assert np.array_equal(cs["support"], fu["support"])
    np.testing.assert_allclose(cs["coef"], fu["coef"], rtol=0, atol=0)


# --------------------------------------------------------------------------
# P6: Phi = I, box average / replication: (P_low) equals Algorithm 2's W x step.
# --------------------------------------------------------------------------
def pin_identity_fold(lib, seed=18):
    """With U replicating over equal blocks of b samples and W averaging them,
    UW is the orthogonal projector onto block-constant vectors; hence OMP on
    y with atoms U d picks the same atoms as OMP on W y with atoms d, and the
    coefficients agree (Section III-C, Step 1 vs Algorithm 2)."""
    import synth
    w = synth.make("c1", batch=256)
    out = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "identity", w.m, None, w.y, None, [4, 4], lib_path=lib)
    up = w.up_maps[0]
    wy = np.zeros((w.batch, 16))
    np.add.at(wy.T, up, w.y.T)
    wy /= 4.0
    low = oracle.omp([16], [64], [w.dicts[0]], [], "identity", 16, None, wy, None, [4], lib_path=lib)
    assert np.array_equal(out["supports"][:, 0, :4], low["support"][:, :4])
    np.testing.assert_allclose(out["coefs"][:, 0, :4], low["coef"][:, :4], rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------
# P7: measurement operators agree with each other.
# --------------------------------------------------------------------------
def pin_operators(lib, seed=19):
    """diag(mask) (mask path) == dense Phi = I restricted to observed rows
    (dense path, M = #observed); an all-ones mask == identity; a dense
    identity Phi == the identity path."""
    import synth
    w = synth.custom([16, 64], [32, 128], batch=24, seed=seed, k_scales=[3, 5], sigma=0.02,
                     phi_kind="mask", dict_kind="model")
    mask_out = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "mask", w.m, None, w.y, w.mask,
                          [3, 5], lib_path=lib)
    for b in range(w.batch):
        obs = np.flatnonzero(w.mask[b])
        phi = np.eye(64)[obs]
        d = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "dense", len(obs), phi, w.y[b:b + 1, obs],
                       None, [3, 5], lib_path=lib)
        assert np.array_equal(d["supports"][0], mask_out["supports"][b])
        np.testing.assert_allclose(d["coefs"][0], mask_out["coefs"][b], rtol=1e-9, atol=1e-12)
    ones = np.ones_like(w.mask)
    a = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "mask", w.m, None, w.x, ones, [3, 5], lib_path=lib)
    b_ = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "identity", w.m, None, w.x, None, [3, 5], lib_path=lib)
    c_ = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "dense", 64, np.eye(64), w.x, None, [3, 5], lib_path=lib)
    assert np.array_equal(a["supports"], b_["supports"]) and np.array_equal(b_["supports"], c_["supports"])
    np.testing.assert_allclose(a["coefs"], b_["coefs"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(c_["coefs"], b_["coefs"], rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------
# Stopping rules: exhausted candidates and dependence.
# --------------------------------------------------------------------------
def pin_stopping(lib, seed=20):
    """K larger than the candidate set is capped (|f(Omega)| = Q K_low); K at
    the rank of the measurement space stops at M atoms; a duplicated atom is
    never selected twice (it is dependent)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((10, 4))
    y = rng.standard_normal(4)
    out = _single(d, y, 8, lib)
    assert int(out["k_used"][0, 0]) == 4                  # rank 4
    r = y - d[out["support"][0, :4]].T @ out["coef"][0, :4]
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(y)
    d2 = np.vstack([d[:3], d[:1] * 2.0])                    # atom 3 parallel to atom 0
    out = _single(d2, d2[0] * 1.5 + d2[1], 4, lib)
    ku = int(out["k_used"][0, 0])
    sup = list(out["support"][0, :ku])
    assert not (0 in sup and 3 in sup)
    import synth
    w = synth.custom([4, 16], [4, 8], batch=8, seed=seed, k_scales=[1, 5], sigma=0.1)
    out = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "identity", w.m, None, w.y, None, [1, 5], lib_path=lib)
    assert np.all(out["k_used"][:, 1] == 2)               # Q * K_low = 2 candidates


# --------------------------------------------------------------------------
# Forced prefix and per-step trace: replaying another solver's choices.
# The near-tie rule that excuses a GPU pick reads the trace (best score,
# runner-up, score of the pick, step-1 maximum), so both are pinned.
# --------------------------------------------------------------------------
FORCED_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "omp_forced.json")


def pin_golden_forced(lib):
    """Hand-worked runs with imposed picks (tests/golden/omp_forced.json):
    supports, coefficients and all four trace values of every step."""
    g = json.load(open(FORCED_GOLDEN))
    for case in g["cases"]:
        k = case["k"]
        forced = np.asarray(case["forced"], dtype=np.int32).reshape(1, 1, k)
        out = _single(case["dict_atoms"], case["y"], k, lib, forced=forced, kstride=k, with_trace=True)
        ku = int(out["k_used"][0, 0])
        assert ku == case["k_used"], (case["name"], ku)
        assert list(out["support"][0, :ku]) == case["support"], (case["name"], out["support"][0])
        np.testing.assert_allclose(out["coef"][0, :ku], case["coef"], rtol=1e-12, atol=1e-12,
                                   err_msg=case["name"])
        tr = out["trace"][0, 0]
        want = np.asarray(case["trace"], dtype=np.float64)
        np.testing.assert_allclose(tr[:len(want)], want, rtol=1e-12, atol=1e-12, err_msg=case["name"])


def _greedy_trace(a, y, k, forced):
    """Independent re-derivation of Algorithm 1 with imposed steps: the residue
    of every step from LAPACK least squares on the support so far, the scores
    of the remaining atoms, and the four trace values."""
    t = a.shape[1]
    nu = np.linalg.norm(a, axis=0)
    sup, rows = [], []
    first = None
    for n in range(k):
        r = y if not sup else _lstsq_residual(a[:, sup], y)[0]
        sc = np.abs(a.T @ r) / nu
        avail = np.ones(t, dtype=bool)
        avail[sup] = False
        order = np.argsort(-np.where(avail, sc, -np.inf), kind="stable")
        best = sc[order[0]]
        runner = sc[order[1]] if avail.sum() > 1 else -1.0
        if first is None:
            first = best
        f = int(forced[n])
        if f >= 0 and not avail[f]:
            rows.append([0.0, 0.0, 0.0, 0.0])
            break
        pick = f if f >= 0 else int(order[0])
        rows.append([best, runner, sc[pick], first])
        sup.append(pick)
    return sup, np.asarray(rows)


def pin_trace_bruteforce(lib, trials=60, seed=24):
    """Random tiny problems with random imposed steps (the runner-up, any
    other remaining atom, or an atom already chosen): the oracle's supports,
    coefficients and trace rows equal an independent re-derivation that
    recomputes every residue with LAPACK least squares."""
    rng = np.random.default_rng(seed)
    for trial in range(trials):
        m, t = int(rng.integers(5, 9)), int(rng.integers(6, 12))
        k = int(rng.integers(2, min(m, t) - 1))
        d = rng.standard_normal((t, m))
        d[rng.integers(0, t)] *= 2.5
        y = rng.standard_normal(m)
        a = d.T
        free, _ = _greedy_trace(a, y, k, [-1] * k)
        forced = np.full(k, -1, dtype=np.int32)
        for n in range(k):
            u = rng.random()
            if u < 0.3:
                forced[n] = int(rng.integers(0, t))          # any atom (maybe chosen already)
            elif u < 0.5 and n == 0:
                nu = np.linalg.norm(a, axis=0)
                forced[n] = int(np.argsort(-np.abs(a.T @ y) / nu, kind="stable")[1])   # runner-up
        sup, rows = _greedy_trace(a, y, k, forced)
        out = _single(d, y, k, lib, forced=forced.reshape(1, 1, k), kstride=k, with_trace=True)
        ku = int(out["k_used"][0, 0])
        assert ku == len(sup), (trial, ku, sup, forced)
        assert list(out["support"][0, :ku]) == sup, (trial, out["support"][0], sup)
        tr = out["trace"][0, 0]
        np.testing.assert_allclose(tr[:len(rows)], rows, rtol=1e-10, atol=1e-12, err_msg=str(trial))
        assert np.all(tr[len(rows):] == 0.0)
        if ku:
            _, beta = _lstsq_residual(a[:, sup], y)
            np.testing.assert_allclose(out["coef"][0, :ku], beta, rtol=1e-9, atol=1e-12)
        # without imposed steps the trace's picked score is its best score
        out0 = _single(d, y, k, lib, with_trace=True)
        assert list(out0["support"][0, :k]) == free
        np.testing.assert_array_equal(out0["trace"][0, 0, :, 0], out0["trace"][0, 0, :, 2])


def pin_forced(lib, seed=21):
    """Forcing the oracle's own choices reproduces it bit for bit; forcing the
    runner-up at the first step of the fine scale gives a trace whose picked
    score is the runner-up's and whose later steps are greedy again (checked
    against LAPACK least squares on the forced prefix)."""
    import synth
    w = synth.make("c2", batch=32)
    base = oracle.omp_cross_scale(w, with_trace=True, lib_path=lib)
    forced = base["supports"].copy()
    again = oracle.omp_cross_scale(w, forced=forced, kstride=forced.shape[2], lib_path=lib)
    assert np.array_equal(again["supports"], base["supports"])
    assert np.array_equal(again["coefs"], base["coefs"])
    S, kst = base["supports"].shape[1], base["supports"].shape[2]
    for b in range(w.batch):
        f = np.full((1, S, kst), -1, dtype=np.int32)
        f[0, 0] = base["supports"][b, 0]                     # keep the coarse scale
        cand = sorted(p * 8 + j for p in base["supports"][b, 0, :base["k_used"][b, 0]] for j in range(8))
        a = np.where(w.mask[b][:, None] != 0, w.dicts[1].T, 0.0)
        nu = np.linalg.norm(a, axis=0)
        sc = np.full(a.shape[1], -1.0)
        sc[cand] = np.abs(a[:, cand].T @ w.y[b]) / nu[cand]
        ru = int(np.argsort(-sc, kind="stable")[1])
        f[0, 1, 0] = ru
        sub = synth.subset(w, [b])
        out = oracle.omp_cross_scale(sub, forced=f, kstride=kst, with_trace=True, lib_path=lib)
        tr = out["trace"][0, 1]
        assert out["supports"][0, 1, 0] == ru
        np.testing.assert_allclose(tr[0, :3], [sc.max(), sc[ru], sc[ru]], rtol=1e-10)
        np.testing.assert_allclose(tr[:, 3][:out["k_used"][0, 1]], sc.max(), rtol=1e-10)
        fine = list(out["supports"][0, 1, :out["k_used"][0, 1]])
        for n in range(1, len(fine)):
            r = _lstsq_residual(a[:, fine[:n]], w.y[b])[0]
            s2 = np.full(a.shape[1], -1.0)
            s2[cand] = np.abs(a[:, cand].T @ r) / nu[cand]
            s2[fine[:n]] = -1.0
            assert s2[fine[n]] >= s2.max() - 1e-12, (b, n)
            np.testing.assert_allclose(tr[n, 2], s2[fine[n]], rtol=1e-9, atol=1e-14)


# --------------------------------------------------------------------------
# Three scales: each scale is greedy over the children of the scale above,
# with effective atoms built from explicit 0/1 upsampling matrices.
# --------------------------------------------------------------------------
def _up_matrix(up, n_coarse):
    u = np.zeros((len(up), n_coarse))
    u[np.arange(len(up)), up] = 1.0
    return u


def pin_three_scales(lib, trials=20, seed=22):
    import synth
    up0, _ = synth.box_map((4, 4), (2, 2))
    up1, _ = synth.box_map((8, 8), (2, 2))
    dims, atoms, ks = [4, 16, 64], [6, 24, 96], [2, 3, 4]
    rng = np.random.default_rng(seed)
    for t in range(trials):
        dicts = [rng.standard_normal((atoms[s], dims[s])) for s in range(3)]
        m = 40
        phi = rng.standard_normal((m, 64)) / np.sqrt(m)
        y = rng.standard_normal((1, m))
        out = oracle.omp(dims, atoms, dicts, [up0, up1], "dense", m, phi, y, None, ks, lib_path=lib)
        u1 = _up_matrix(up1, 16)
        u0 = u1 @ _up_matrix(up0, 4)
        eff = [phi @ u0 @ dicts[0].T, phi @ u1 @ dicts[1].T, phi @ dicts[2].T]
        prev = None
        for s in range(3):
            a = eff[s]
            sup = list(out["supports"][0, s, :out["k_used"][0, s]])
            if prev is None:
                cand = list(range(atoms[s]))
            else:
                q = atoms[s] // atoms[s - 1]
                cand = sorted(p * q + j for p in prev for j in range(q))
            assert len(sup) == min(ks[s], len(cand))
            nu = np.linalg.norm(a, axis=0)
            for n, pick in enumerate(sup):
                assert pick in cand
                r = y[0] if n == 0 else _lstsq_residual(a[:, sup[:n]], y[0])[0]
                sc = np.full(atoms[s], -1.0)
                sc[cand] = np.abs(a[:, cand].T @ r) / nu[cand]
                sc[sup[:n]] = -1
                assert sc[pick] >= sc.max() - 1e-12, (s, n)
            res, beta = _lstsq_residual(a[:, sup], y[0])
            np.testing.assert_allclose(out["coefs"][0, s, :len(sup)], beta, rtol=1e-9, atol=1e-12)
            prev = sup
        xh = dicts[2][prev].T @ out["coef"][0, :len(prev)]
        np.testing.assert_allclose(out["xhat"][0], xh, rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------
# Per-patch operators chosen from a set (location-dependent measurements).
# --------------------------------------------------------------------------
def pin_phases(lib, seed=25):
    """A batch measured with several dense operators, each patch with its
    own: the phased run equals, patch for patch and bit for bit, a plain run
    of each phase's patches with that phase's single operator; and operators
    diag(m_p) give exactly the per-patch mask run with masks m_p."""
    import synth
    rng = np.random.default_rng(seed)
    w = synth.custom([16, 64], [32, 256], batch=90, seed=seed, k_scales=[3, 6], sigma=0.02,
                     phi_kind="dense", m=40)
    P = 3
    phis = np.stack([w.phi] + [rng.standard_normal(w.phi.shape) / np.sqrt(40) for _ in range(P - 1)])
    ph = rng.integers(0, P, size=w.batch).astype(np.int32)
    y = w.y
    out = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "dense", w.m, phis, y, None, w.k_scales,
                     phase=ph, lib_path=lib)
    for p in range(P):
        idx = np.where(ph == p)[0]
        ref = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "dense", w.m, phis[p], y[idx], None,
                         w.k_scales, lib_path=lib)
        for key in ("supports", "coefs", "k_used", "xhat"):
            assert np.array_equal(out[key][idx], ref[key]), (p, key)
    # diag(mask) operators = the mask path
    masks = rng.integers(0, 2, size=(P, 64)).astype(np.uint8)
    dphi = np.stack([np.diag(m.astype(np.float64)) for m in masks])
    x = w.x
    ph2 = rng.integers(0, P, size=w.batch).astype(np.int32)
    yd = x * masks[ph2]
    outd = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "dense", 64, dphi, yd, None, w.k_scales,
                      phase=ph2, lib_path=lib)
    outm = oracle.omp(w.dims, w.atoms, w.dicts, w.up_maps, "mask", 64, None, yd, masks[ph2], w.k_scales,
                      lib_path=lib)
    for key in ("supports", "k_used"):
        assert np.array_equal(outd[key], outm[key]), key
    assert np.allclose(outd["coefs"], outm["coefs"], rtol=0, atol=1e-12 * np.abs(outm["coefs"]).max())


ALL_PINS = [pin_phases, pin_golden, pin_bruteforce_greedy, pin_bruteforce_cross_scale, pin_exact_recovery,
            pin_exact_recovery_cross_scale, pin_orthonormal, pin_invariants, pin_reductions,
            pin_identity_fold, pin_operators, pin_stopping, pin_forced, pin_golden_forced,
             pin_trace_bruteforce, pin_three_scales]
