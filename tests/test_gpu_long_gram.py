"""The long-vector kernel's Gram mode (patches with at most 64 candidates)
against the FP64 oracle at its edges: patches with nothing observed, with
fewer observed samples than the sparsity (the rank bound), per-patch fine
sparsity from zero to above the candidate count, and children that are
exact or near duplicates of each other (the dependence test of Algorithm
1's merge on FP64 Gram entries).  24x24 patches over 12x12 under a
per-patch pixel mask: scale 0 holds 64 candidates over 144 coordinates
(2x2 blocks of fine samples, weights sqrt(count)), scale 1 the children of
the coarse support over 576 coordinates (one fine sample each).
"""
import dataclasses

import numpy as np
import pytest

from test_gpu_long import _kernels, long_workload
from test_gpu_parity import check_cross
from paper_1511_05174_amd import cspd

pytestmark = pytest.mark.gpu


def _gram_mode_ran(w):
    labels = _kernels(cspd.plan_from_workload(w), w)
    assert any(l.startswith("omp_long<f32,gram,") and l.endswith(":s1") for l in labels), labels
    assert any(l.startswith("omp_long<f32,gram,") and l.endswith(":s0") for l in labels), labels


def test_gram_mode_masks_and_ragged_sparsity():
    w = long_workload("img24", 240, seed=41, atoms=(64, 512), ks=(2, 6), phi_kind="mask")
    rng = np.random.default_rng(5)
    mask = w.mask.copy()
    mask[0:6] = 0                                   # nothing observed
    mask[6:12, :288] = 0                            # the top half hidden
    for b in range(12, 18):                         # three samples: at most three atoms
        mask[b] = 0
        mask[b, rng.choice(576, 3, replace=False)] = 1
    kf = rng.integers(0, 17, size=w.batch).astype(np.int32)   # 16 candidates at scale 1
    kf[18:24] = 0
    kf[24:30] = 16
    # measurements at every sample (the workload's own are zero where its
    # mask was zero, which would make every score tie at rounding noise)
    y = w.x + 0.01 * rng.standard_normal(w.x.shape)
    w = dataclasses.replace(w, mask=mask, k_fine=kf, y=y)
    print(f"gram mode: B {w.batch}, k_fine {kf.min()}..{kf.max()}, observed "
          f"{int(mask.sum(1).min())}..{int(mask.sum(1).max())} of 576", flush=True)
    out, rep = check_cross(w)
    assert np.all(out["k_used"][0:6] == 0)
    assert np.all(out["k_used"][12:18] <= 3)
    assert np.all(out["k_used"][18:24] == 0)
    _gram_mode_ran(w)


def test_gram_mode_duplicate_children():
    """Child 1 of every parent is child 0 again and child 2 differs from it
    by 2^-9 in one sample; measurements mix child 0 and child 2 of one
    parent with a third atom, so the picks meet the duplicates."""
    w = long_workload("img24", 200, seed=42, atoms=(64, 512), ks=(3, 6), phi_kind="mask")
    q = 8
    d1 = w.dicts[1].copy()
    for p in range(w.atoms[0]):
        d1[p * q + 1] = d1[p * q]
        d1[p * q + 2] = d1[p * q]
        d1[p * q + 2, (7 * p) % d1.shape[1]] += 2.0 ** -9
    rng = np.random.default_rng(9)
    par = rng.integers(0, w.atoms[0], size=w.batch)
    other = rng.integers(0, w.atoms[1], size=w.batch)
    y = d1[par * q] - 0.8 * d1[par * q + 2] + 0.5 * d1[other] + 0.01 * rng.standard_normal((w.batch, d1.shape[1]))
    w = dataclasses.replace(w, dicts=[w.dicts[0], d1], y=y)
    out, rep = check_cross(w, max_excused=1 + w.batch // 100)
    # an exact duplicate never joins a support that holds its twin
    sup = out["support"]
    for b in range(w.batch):
        s = set(int(a) for a in sup[b] if a >= 0)
        for a in s:
            if a % q == 1:
                assert a - 1 not in s, (b, sorted(s))
    _gram_mode_ran(w)
