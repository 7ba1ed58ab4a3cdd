"""Learning cross-scale dictionaries (Section III-E) with the library's kernels.

Step 1: K-SVD on the down-sampled training set gives D_low (and, as a
by-product, the coarse supports).  Step 2: K-SVD whose sparse-approximation
step is zero-tree OMP -- every signal's fine support stays inside the
children of its coarse support -- gives D_high.  The sparse approximation
runs on ``cspd_omp_full`` / ``cspd_omp_cross_scale`` and the dictionary
update on ``cspd_ksvd_update``; this module only sequences them (and builds
the plans, which take host FP64 dictionaries).

Initialisation (Section III-G, heuristics 1 and 2): D_low from randomly
picked training signals; the children of coarse atom k from randomly picked
training signals whose coarse support holds k (all signals when fewer than Q
do).  Replacement (heuristics 3 and 4): after each update sweep an atom that
no training signal used is replaced by the least represented signal -- the
largest representation error left by that iteration's sparse approximation,
ties to the lower index, each signal taken once per sweep -- drawn, for an
atom of D_high, from the signals whose coarse support holds its parent (all
signals when none does); the new atom is that signal at unit norm.
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


def replace_unused(d: np.ndarray, x: np.ndarray, support: np.ndarray, err: np.ndarray,
                   coarse: Optional[np.ndarray] = None, q: int = 1):
    """Heuristics 3 and 4: atoms (rows of d) that no support used, in index
    order, each take the least represented signal not yet taken (for a child
    atom, among the signals whose coarse support holds its parent, else all).
    Returns (d', list of replaced atoms)."""
    d = np.array(d, copy=True)
    used = np.zeros(d.shape[0], dtype=bool)
    used[support[support >= 0].astype(np.int64)] = True
    free = np.ones(x.shape[0], dtype=bool)
    done = []
    for a in np.nonzero(~used)[0]:
        cand = np.arange(x.shape[0])
        if coarse is not None:
            holds = np.nonzero(np.any(coarse == a // q, axis=1))[0]
            if holds.size:
                cand = holds
        cand = cand[free[cand]]
        if cand.size == 0:
            continue
        j = int(cand[np.argmax(err[cand])])    # argmax: first of equal values
        nrm = float(np.linalg.norm(x[j]))
        if nrm <= 0.0:
            continue
        d[a] = x[j] / nrm
        free[j] = False
        done.append(int(a))
    return d, done


def ksvd(x: np.ndarray, d0: np.ndarray, k: int, iters: int, timings: Optional[list] = None,
         replace: bool = True, replaced: Optional[list] = None):
    """Plain K-SVD (Algorithm 1 as the sparse-approximation step) on the
    device.  x: (P, N) signals, d0: (T, N) initial atoms.  Returns (D, support,
    coef) after the last sweep; `timings` collects (coding_s, update_s) per
    iteration, `replaced` the atoms heuristic 3 replaced in each."""
    torch = cspd._torch()
    dev = torch.device("cuda", 0)
    X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    xf = X.cpu().numpy().astype(np.float64)
    D = torch.from_numpy(np.ascontiguousarray(d0, dtype=np.float32)).to(dev)
    st = None
    for _ in range(iters):
        D, st = ksvd_step(X, xf, D, k, replace)
        if replaced is not None:
            replaced.append(st["replaced"])
        if timings is not None:
            timings.append((st["coding_s"], st["update_s"]))
    return D.cpu().numpy(), st["support"], st["coef_updated"]


def ksvd_step(X, xf: np.ndarray, D, k: int, replace: bool = True):
    """One plain K-SVD iteration: Algorithm 1 coding of the signals X (device,
    FP32; xf the same values in FP64 on the host) over the atoms D (device
    rows, updated in place or replaced), the update sweep, then heuristic 3.
    Returns (D, stats): the coding's supports and coefficients, the
    coefficients after the sweep, the replaced atoms and the times."""
    torch = cspd._torch()
    plan = _plan([X.shape[1]], [D.shape[0]], [D.cpu().numpy().astype(np.float64)], [], max(k, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sup, coef, _, xh = cspd.cspd_omp_full(plan, X, None, None, k, want_xhat=replace)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = {"support": sup.cpu().numpy(), "coef": coef.cpu().numpy()}
    cspd.cspd_ksvd_update(X, D, sup, coef)
    torch.cuda.synchronize()
    st["coding_s"], st["update_s"] = t1 - t0, time.perf_counter() - t1
    st["coef_updated"] = coef.cpu().numpy()
    st["replaced"] = []
    if replace:
        err = np.linalg.norm(xf - xh.cpu().numpy().astype(np.float64), axis=1)
        dn, done = replace_unused(D.cpu().numpy(), xf, st["support"], err)
        if done:
            D = torch.from_numpy(np.ascontiguousarray(dn, dtype=np.float32)).to(X.device)
        st["replaced"] = done
    cspd.cspd_plan_destroy(plan)
    return D, st


def cross_scale_step(X, xf: np.ndarray, d_low: np.ndarray, D, up_map: np.ndarray, n_low: int, q: int,
                     k_low: int, k_high: int, replace: bool = True):
    """One iteration of step 2 (Section III-E): zero-tree OMP of the signals
    X (device, FP32; xf the same values in FP64 on the host) over D_low and
    D_high = D (device rows, updated in place or replaced), the K-SVD update
    sweep, then heuristic 4.  Returns (D, stats) with the supports, the
    coefficients, the coarse supports and the replaced atoms in stats."""
    torch = cspd._torch()
    t_low = d_low.shape[0]
    plan = _plan([n_low, X.shape[1]], [t_low, t_low * q],
                 [d_low.astype(np.float64), D.cpu().numpy().astype(np.float64)], [up_map], max(k_low, k_high))
    sc = torch.empty((X.shape[0], max(k_low, 1)), dtype=torch.int32, device=X.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sup, coef, _, xh = cspd.cspd_omp_cross_scale(plan, X, None, [k_low], None, k_high, want_xhat=replace,
                                                 support_coarse=sc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = {"support": sup.cpu().numpy(), "coef": coef.cpu().numpy(), "coarse": sc.cpu().numpy()[:, :k_low]}
    cspd.cspd_ksvd_update(X, D, sup, coef)
    torch.cuda.synchronize()
    st["coding_s"], st["update_s"] = t1 - t0, time.perf_counter() - t1
    st["replaced"] = []
    if replace:
        # heuristic 4: Omega_k = the signals whose coarse support holds k
        err = np.linalg.norm(xf - xh.cpu().numpy().astype(np.float64), axis=1)
        dn, done = replace_unused(D.cpu().numpy(), xf, st["support"], err, coarse=st["coarse"], q=q)
        if done:
            D = torch.from_numpy(np.ascontiguousarray(dn, dtype=np.float32)).to(X.device)
        st["replaced"] = done
    cspd.cspd_plan_destroy(plan)
    return D, st


def cross_scale(x: np.ndarray, up_map: np.ndarray, n_low: int, t_low: int, q: int, k_low: int, k_high: int,
                iters_low: int, iters_high: int, seed: int = 0, timings: Optional[dict] = None,
                replace: bool = True):
    """Section III-E, steps 1 and 2.  Returns (D_low, D_high) as (T, N) atom
    rows; `timings` gets per-iteration (coding_s, update_s) lists under
    'low' and 'high' and the replaced atoms under 'replaced_low' and
    'replaced_high'."""
    torch = cspd._torch()
    rng = np.random.default_rng(seed)
    xl = downsample(x, up_map, n_low)
    d_low0 = _unit_rows(xl[rng.choice(len(xl), size=t_low, replace=False)])
    tl = [] if timings is not None else None
    rl = []
    d_low, sup_low, _ = ksvd(xl, d_low0, k_low, iters_low, tl, replace=replace, replaced=rl)
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
    xf = X.cpu().numpy().astype(np.float64)
    D = torch.from_numpy(np.ascontiguousarray(d_high, dtype=np.float32)).to(dev)
    th, rh = [], []
    for _ in range(iters_high):
        D, st = cross_scale_step(X, xf, d_low, D, up_map, n_low, q, k_low, k_high, replace)
        th.append((st["coding_s"], st["update_s"]))
        rh.append(st["replaced"])
    if timings is not None:
        timings["low"] = tl
        timings["high"] = th
        timings["replaced_low"] = rl
        timings["replaced_high"] = rh
    return d_low, D.cpu().numpy()
