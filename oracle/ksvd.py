"""Dictionary update of K-SVD as used to learn the cross-scale dictionaries
(Section III-E: K-SVD on the down-sampled training set for D_low, then the
same update with the sparse-approximation step restricted to the children of
the coarse support for D_high) -- test infrastructure only.

Plain numpy, FP64, one atom after another in index order so that it can be
checked by eye against the algorithm.  It shares no code with the HIP
library.  The sparse-approximation step itself is the OMP oracle
(``oracle.omp``); this module only holds the dictionary update and the
initialisation heuristic of Section III-G.

Readings (the paper names K-SVD and leaves these details to it):
  * atoms are updated in index order; each update uses the coefficients and
    atoms as left by the previous one (the sequential K-SVD update);
  * the new atom is the leading left singular vector of the restricted error
    matrix E_k, with its sign chosen so that it does not point away from the
    old atom; the users' coefficients become E_k^T d;
  * an atom that no training signal uses keeps its value during the sweep;
    afterwards the replacement heuristics 3 and 4 of Section III-G may
    replace it (``replace_unused``): by the least represented training
    signal -- the one with the largest representation error
    ||x_j - x_hat_j|| left by the sparse-approximation step of the same
    iteration (ties to the lower index) -- drawn, for an atom of D_high,
    from the signals whose coarse support holds the atom's parent (all
    signals when none does); unused atoms are visited in index order and
    each takes a signal not taken before in the same sweep; the new atom is
    that signal scaled to unit norm.
"""
from __future__ import annotations

import numpy as np


def residual(X: np.ndarray, D: np.ndarray, support: np.ndarray, coef: np.ndarray) -> np.ndarray:
    """R = X - D S for signals X (P x N), atoms D (T x N), supports and
    coefficients (P x kstride, -1 = unused slot)."""
    R = np.array(X, dtype=np.float64, copy=True)
    for p in range(X.shape[0]):
        for j in range(support.shape[1]):
            a = int(support[p, j])
            if a >= 0:
                R[p] -= coef[p, j] * D[a]
    return R


def update(X: np.ndarray, D: np.ndarray, support: np.ndarray, coef: np.ndarray):
    """One sweep of the K-SVD dictionary update.  Returns (D', coef', R) with
    R the residual after the sweep; inputs are not modified."""
    D = np.array(D, dtype=np.float64, copy=True)
    coef = np.array(coef, dtype=np.float64, copy=True)
    R = residual(X, D, support, coef)
    T = D.shape[0]
    for k in range(T):
        users = np.argwhere(support == k)            # (patch, slot) pairs, patch order
        if users.shape[0] == 0:
            continue
        rows, slots = users[:, 0], users[:, 1]
        s_old = coef[rows, slots]
        E = R[rows] + np.outer(s_old, D[k])           # users x N: the error without atom k
        U, sig, Vt = np.linalg.svd(E.T, full_matrices=False)
        d = U[:, 0]
        if d @ D[k] < 0:
            d = -d
        s_new = E @ d
        D[k] = d
        coef[rows, slots] = s_new
        R[rows] = E - np.outer(s_new, d)
    return D, coef, R


def init_children(X: np.ndarray, coarse_support: np.ndarray, q: int, t_low: int, rng) -> np.ndarray:
    """Initial D_high (Section III-G, heuristic 2): the Q children of coarse
    atom k are distinct training signals drawn at random from those whose
    coarse support contains k (unit norm); when fewer exist, from all."""
    n = X.shape[1]
    D = np.zeros((t_low * q, n))
    allp = np.arange(X.shape[0])
    for k in range(t_low):
        pool = np.nonzero(np.any(coarse_support == k, axis=1))[0]
        if pool.size < q:
            pool = allp
        pick = rng.choice(pool, size=q, replace=False)
        for c, p in enumerate(pick):
            v = X[p] / max(np.linalg.norm(X[p]), 1e-300)
            D[k * q + c] = v
    return D


def replace_unused(D: np.ndarray, X: np.ndarray, support: np.ndarray, err: np.ndarray,
                   coarse_support: np.ndarray = None, q: int = 1):
    """Heuristics 3 and 4 of Section III-G.  D (T x N) atoms after the update
    sweep, X (P x N) training signals, support (P x kstride) the supports the
    sweep used, err (P,) every signal's representation error after the
    sparse-approximation step.  With coarse_support (P x k_low) and q, atom a
    is a child of coarse atom a // q and its candidates are the signals
    whose coarse support holds that parent.  Returns (D', replaced atoms)."""
    D = np.array(D, dtype=np.float64, copy=True)
    used = np.zeros(D.shape[0], dtype=bool)
    s = support[support >= 0]
    used[s.astype(np.int64)] = True
    taken = np.zeros(X.shape[0], dtype=bool)
    replaced = []
    for a in range(D.shape[0]):
        if used[a]:
            continue
        if coarse_support is not None:
            pool = np.nonzero(np.any(coarse_support == a // q, axis=1))[0]
            if pool.size == 0:
                pool = np.arange(X.shape[0])
        else:
            pool = np.arange(X.shape[0])
        pool = pool[~taken[pool]]
        if pool.size == 0:
            continue
        # the largest error, the lowest index among equal ones
        j = int(pool[np.argmax(err[pool])])
        nrm = np.linalg.norm(X[j])
        if nrm <= 0.0:
            continue
        D[a] = X[j] / nrm
        taken[j] = True
        replaced.append(a)
    return D, replaced
