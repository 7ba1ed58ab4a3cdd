"""Whole-signal patch processing around the OMP hot path (Section IV): cut a
signal (image, video, light field) into overlapping patches, and put patch
estimates back together by averaging every estimate that covers a sample.

Test infrastructure only (like the rest of ``oracle``): plain numpy,
FP64 for the averaging, loops over the patch grid so that each step can be
checked by eye.  It shares no code with the HIP library.

Conventions (the paper processes overlapping patches, e.g. 24 x 24 image
patches with an overlap of 18 samples, and leaves the grid and the
averaging unstated; the readings used here):
  * the patch grid of each axis starts at 0 and steps by the stride; when the
    last regular position does not reach the end of the axis, one more
    position, aligned to the end, is added, so every sample is covered;
  * patches are numbered row-major over the grid (first axis slowest), and a
    patch is vectorised row-major over its own axes (image (y, x), video
    (t, y, x), light field (u, v, y, x));
  * a sample's estimate is the plain mean of the estimates of every patch
    that covers it.
"""
from __future__ import annotations

import itertools
from typing import List, Sequence

import numpy as np


def grid_positions(dim: int, patch: int, stride: int) -> List[int]:
    """Start positions of the patches along one axis."""
    if not (1 <= patch <= dim) or stride < 1:
        raise ValueError(f"patch {patch}, stride {stride} on an axis of {dim}")
    pos = list(range(0, dim - patch + 1, stride))
    if pos[-1] != dim - patch:
        pos.append(dim - patch)
    return pos


def patch_grid(dims: Sequence[int], patch: Sequence[int], stride: Sequence[int]) -> List[List[int]]:
    return [grid_positions(d, p, s) for d, p, s in zip(dims, patch, stride)]


def extract(signal: np.ndarray, patch: Sequence[int], stride: Sequence[int]) -> np.ndarray:
    """(number of patches) x (patch volume) array of the signal's patches."""
    grids = patch_grid(signal.shape, patch, stride)
    rows = []
    for start in itertools.product(*grids):
        sl = tuple(slice(s, s + p) for s, p in zip(start, patch))
        rows.append(np.asarray(signal[sl]).reshape(-1))
    return np.stack(rows)


def aggregate(patches: np.ndarray, dims: Sequence[int], patch: Sequence[int],
              stride: Sequence[int]) -> np.ndarray:
    """Mean over the covering patches of their estimates, in FP64."""
    grids = patch_grid(dims, patch, stride)
    acc = np.zeros(tuple(dims), dtype=np.float64)
    cnt = np.zeros(tuple(dims), dtype=np.float64)
    for i, start in enumerate(itertools.product(*grids)):
        sl = tuple(slice(s, s + p) for s, p in zip(start, patch))
        acc[sl] += np.asarray(patches[i], dtype=np.float64).reshape(tuple(patch))
        cnt[sl] += 1.0
    return acc / cnt
