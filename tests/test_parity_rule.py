"""The GPU-vs-oracle comparison itself (CPU only): results planted from the
oracle's own runs must be judged as the near-tie rule says -- an identical run
passes, a far-off pick is a mismatch, a pick within the tie tolerance is
excused (and counted), and a small coefficient that is off is caught entry by
entry."""
import numpy as np
import pytest

import oracle
import parity
import synth


def _gpu_like(res, S):
    """Oracle outputs arranged as a GPU call returns them (finest scale)."""
    return (res["supports"].copy(), res["coef"].copy(), res["k_fine_used"].copy(), res["xhat"].copy())


def test_identical_run_passes():
    w = synth.make("c2", batch=64)
    res = oracle.omp_cross_scale(w)
    sup, coef, ku, xh = _gpu_like(res, w.n_scales)
    rep = parity.compare(w, sup, coef, ku, xh)
    assert not rep.mismatched and rep.excused == 0
    assert rep.coef_rel_max == 0.0 and rep.xhat_rel_max == 0.0
    rep.check(1e-5, 1e-5)


def test_small_coefficient_caught_entry_by_entry():
    w = synth.make("c2", batch=32)
    res = oracle.omp_cross_scale(w)
    sup, coef, ku, xh = _gpu_like(res, w.n_scales)
    b = 3
    k = int(ku[b])
    i = int(np.argmin(np.abs(coef[b, :k])))
    amax = np.max(np.abs(coef[b, :k]))
    coef[b, i] += 3e-5 * amax
    rep = parity.compare(w, sup, coef, ku, xh)
    assert rep.coef_rel_max == pytest.approx(3e-5, rel=1e-6)
    assert rep.worst_coef_patch == b
    with pytest.raises(AssertionError):
        rep.check(1e-5, 1e-5)


def test_far_pick_is_a_mismatch_and_reported():
    w = synth.make("c2", batch=16)
    base = oracle.omp_cross_scale(w, with_trace=True)
    b = 5
    # impose the fine scale's runner-up at its first step: gap well above 1e-6
    tr = base["trace"][b, 1, 0]
    assert (tr[0] - tr[1]) / tr[3] > 1e-4
    S, kst = base["supports"].shape[1:]
    f = np.full((w.batch, S, kst), -1, dtype=np.int32)
    f[:, 0] = base["supports"][:, 0]
    sub = synth.subset(w, [b])
    # runner-up: the second best child of the coarse support at step 1
    cand = sorted(p * 8 + j for p in base["supports"][b, 0, :4] for j in range(8))
    a = np.where(w.mask[b][:, None] != 0, w.dicts[1].T, 0.0)
    sc = np.full(a.shape[1], -1.0)
    sc[cand] = np.abs(a[:, cand].T @ w.y[b]) / np.linalg.norm(a[:, cand], axis=0)
    ru = int(np.argsort(-sc, kind="stable")[1])
    f1 = f[b:b + 1].copy()
    f1[0, 1, 0] = ru
    other = oracle.omp_cross_scale(sub, forced=f1, kstride=kst)
    sup, coef, ku, xh = _gpu_like(base, S)
    sup[b] = other["supports"][0]
    coef[b] = other["coef"][0]
    xh[b] = other["xhat"][0]
    rep = parity.compare(w, sup, coef, ku, xh)
    assert rep.mismatched == [b]
    s, n, gap = rep.detail[b]
    assert (s, n) == (1, 0) and gap > 1e-4
    assert rep.xhat_rel_max_mismatched > 0
    with pytest.raises(AssertionError):
        rep.check(1e-5, 1e-5)


def test_near_tie_is_excused_and_counted():
    # two atoms that differ by 1e-9 in direction: whichever the oracle picks,
    # the other is within the tie tolerance
    rng = np.random.default_rng(3)
    d = rng.standard_normal((12, 8))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    y = np.stack([rng.standard_normal(8) for _ in range(6)])
    d[7] = d[2] + 1e-9 * rng.standard_normal(8)
    d[7] /= np.linalg.norm(d[7])
    y[:, :] += 4.0 * d[2]                         # make atom 2 / 7 the first pick
    w = synth.custom([8], [12], batch=6, seed=1, k_scales=[3], sigma=0.0)
    import dataclasses
    w = dataclasses.replace(w, dicts=[d], y=y, x=y, mask=None, phi_kind="identity", m=8, up_maps=[])
    base = oracle.omp_cross_scale(w, with_trace=True)
    first = base["supports"][:, 0, 0]
    assert set(first.tolist()) <= {2, 7}
    swapped = np.where(first == 2, 7, 2).astype(np.int32)
    f = np.full((w.batch, 1, 3), -1, dtype=np.int32)
    f[:, 0, 0] = swapped
    other = oracle.omp_cross_scale(w, forced=f, kstride=3)
    rep = parity.compare(w, other["supports"], other["coef"], other["k_fine_used"], other["xhat"])
    assert not rep.mismatched
    assert rep.excused == w.batch and 0 < rep.worst_tie_gap < 1e-6
    rep.check(1e-5, 1e-5, max_excused=w.batch)
    with pytest.raises(AssertionError):
        rep.check(1e-5, 1e-5, max_excused=w.batch - 1)
