"""Learning cross-scale dictionaries (Section IV) with the library's kernels.

Step 1: K-SVD on the down-sampled training set gives D_low (and, as a
by-product, the coarse supports).  Step 2: K-SVD whose sparse-approximation
step is zero-tree OMP -- every signal's fine support stays inside the
children of its coarse support -- gives D_high.  The sparse approximation
runs on ``cspd_omp_full`` / ``cspd_omp_cross_scale`` and the dictionary
update on ``cspd_ksvd_update``; this module only sequences them (and builds
the plans, which take host FP64 dictionaries).

Initialisation (Section IV-B): D_low from randomly picked training signals;
the children of coarse atom k from randomly picked training signals whose
coarse support holds k (all signals when fewer than Q do).  Atoms without
users keep their value.
"""
from __future__ import annotations

import time
from typing import Optional

import numpy as np

from . import cspd


def downsample(x: np.ndarray, up_map: np.ndarray, n_low: int) -> np.ndarray:
    """W x: the block mean of every coarse coordinate (up_map[j] = the coarse
    coordinate fine coordinate j belongs to)."""
    cnt = np.bincount(up_map, minlength=n_low).astype(np.float64)
    out = np.zeros((x.shape[0], n_low))
    for j, c in enumerate(up_map):
        out[:, c] += x[:, j]
    return out / cnt


def _unit_rows(a: np.ndarray) -> np.ndarray:
    return a / np.maximum(np.linalg.norm(a, axis=1, keepdims=True), 1e-30)


def _plan(dims, atoms, dicts, up_maps, k_max):
    return cspd.cspd_plan(dims, atoms, dicts, up_maps, "identity", dims[-1], None, dtype="f32", k_max=k_max)


def ksvd(x: np.ndarray, d0: np.ndarray, k: int, iters: int, timings: Optional[list] = None):
    """Plain K-SVD (Algorithm 1 as the sparse-approximation step) on the
    device.  x: (P, N) signals, d0: (T, N) initial atoms.  Returns (D, support,
    coef) after the last sweep; `timings` collects (coding_s, update_s) per
    iteration."""
    torch = cspd._torch()
    dev = torch.device("cuda", 0)
    X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    D = torch.from_numpy(np.ascontiguousarray(d0, dtype=np.float32)).to(dev)
    sup = coef = None
    for _ in range(iters):
        plan = _plan([x.shape[1]], [d0.shape[0]], [D.cpu().numpy().astype(np.float64)], [], max(k, 1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sup, coef, _, _ = cspd.cspd_omp_full(plan, X, None, None, k, want_xhat=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cspd.cspd_ksvd_update(X, D, sup, coef)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if timings is not None:
            timings.append((t1 - t0, t2 - t1))
        cspd.cspd_plan_destroy(plan)
    return D.cpu().numpy(), sup.cpu().numpy(), coef.cpu().numpy()


def cross_scale(x: np.ndarray, up_map: np.ndarray, n_low: int, t_low: int, q: int, k_low: int, k_high: int,
                iters_low: int, iters_high: int, seed: int = 0, timings: Optional[dict] = None):
    """Section IV-A, steps 1 and 2.  Returns (D_low, D_high) as (T, N) atom
    rows; `timings` gets per-iteration (coding_s, update_s) lists under
    'low' and 'high'."""
    torch = cspd._torch()
    rng = np.random.default_rng(seed)
    xl = downsample(x, up_map, n_low)
    d_low0 = _unit_rows(xl[rng.choice(len(xl), size=t_low, replace=False)])
    tl = [] if timings is not None else None
    d_low, sup_low, _ = ksvd(xl, d_low0, k_low, iters_low, tl)
    # children of coarse atom k from the signals that use it
    d_high = np.zeros((t_low * q, x.shape[1]))
    allp = np.arange(len(x))
    for k in range(t_low):
        pool = np.nonzero(np.any(sup_low == k, axis=1))[0]
        if pool.size < q:
            pool = allp
        d_high[k * q:(k + 1) * q] = x[rng.choice(pool, size=q, replace=False)]
    d_high = _unit_rows(d_high)
    dev = torch.device("cuda", 0)
    X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    D = torch.from_numpy(np.ascontiguousarray(d_high, dtype=np.float32)).to(dev)
    th = []
    for _ in range(iters_high):
        plan = _plan([n_low, x.shape[1]], [t_low, t_low * q],
                     [d_low.astype(np.float64), D.cpu().numpy().astype(np.float64)], [up_map],
                     max(k_low, k_high))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sup, coef, _, _ = cspd.cspd_omp_cross_scale(plan, X, None, [k_low], None, k_high, want_xhat=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cspd.cspd_ksvd_update(X, D, sup, coef)
        torch.cuda.synchronize()
        th.append((t1 - t0, time.perf_counter() - t1))
        cspd.cspd_plan_destroy(plan)
    if timings is not None:
        timings["low"] = tl
        timings["high"] = th
    return d_low, D.cpu().numpy()
