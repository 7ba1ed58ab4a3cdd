"""Compare a GPU run with the FP64 oracle, patch by patch.

Supports are compared step by step in selection order, at every scale.  At
the first step where they differ, the oracle is re-run with the GPU's picks
forced up to and including that step (its trace then holds, in FP64, the
score of its own best atom and of the GPU's pick).  The divergence is
excused as a near-tie when

    (best score - score of the GPU's pick) / (largest score at step 1 of
    that scale) < tie_tol

and the comparison continues against the replayed oracle; otherwise the
patch is a mismatch.  Coefficients and reconstructions are then compared
with the (replayed) oracle, norm-wise per patch.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import oracle


@dataclass
class Report:
    patches: int
    mismatched: list = field(default_factory=list)     # patch ids with an unexcused divergence
    excused: int = 0                                   # near-ties excused
    k_used_diff: int = 0
    coef_rel_max: float = 0.0
    xhat_rel_max: float = 0.0
    worst_tie_gap: float = 0.0

    def summary(self):
        return (f"patches={self.patches} mismatched={len(self.mismatched)} excused={self.excused} "
                f"coef_rel_max={self.coef_rel_max:.3e} xhat_rel_max={self.xhat_rel_max:.3e} "
                f"worst_excused_gap={self.worst_tie_gap:.3e}")


def gpu_scales(w, support, k_used, support_coarse=None, k_scale=None):
    """Arrange GPU outputs like the oracle's (B, S, kstride) supports."""
    B = support.shape[0]
    S = w.n_scales
    kstride = max([support.shape[1]] + list(k_scale or []))
    sup = np.full((B, S, kstride), -1, dtype=np.int32)
    sup[:, S - 1, :support.shape[1]] = support
    if support_coarse is not None and S > 1:
        off = 0
        for s in range(S - 1):
            sup[:, s, :k_scale[s]] = support_coarse[:, off:off + k_scale[s]]
            off += k_scale[s]
    return sup


def compare(w, gpu_sup, gpu_coef, gpu_kused, gpu_xhat=None, full=False, k_scales=None,
            tie_tol=1e-6, max_rounds=8, coef_k=None):
    """gpu_sup: (B, S, kstride) as from gpu_scales (coarse rows that were not
    recorded stay -1 and are then not compared)."""
    B = gpu_sup.shape[0]
    S = w.n_scales
    kstride = gpu_sup.shape[2]
    ks = list(k_scales if k_scales is not None else w.k_scales)
    rep = Report(patches=B)
    scales = [S - 1] if full else list(range(S))
    have = [s == S - 1 or bool(np.any(gpu_sup[:, s] >= 0)) for s in range(S)]
    forced = np.full((B, S, kstride), -1, dtype=np.int32)
    pending = {}                      # patch -> (scale, step) whose gap must be checked
    final = {}
    active = np.arange(B)
    for _ in range(max_rounds + 1):
        if active.size == 0:
            break
        sub = _subset(w, active)
        res = oracle.omp(sub.dims, sub.atoms, sub.dicts, sub.up_maps, sub.phi_kind, sub.m, sub.phi,
                         sub.y, sub.mask, ks, k_fine=sub.k_fine, full=full, forced=forced[active],
                         kstride=kstride, with_trace=True)
        nxt = []
        for ii, b in enumerate(active):
            b = int(b)
            start = (0, 0)
            if b in pending:
                s, n = pending.pop(b)
                if res["k_used"][ii, s] <= n:
                    rep.mismatched.append(b)      # the GPU's pick is not available / dependent
                    continue
                tr = res["trace"][ii, s, n]
                gap = (tr[0] - tr[2]) / tr[3] if tr[3] > 0 else np.inf
                if not gap < tie_tol:
                    rep.mismatched.append(b)
                    continue
                rep.excused += 1
                rep.worst_tie_gap = max(rep.worst_tie_gap, float(gap))
                start = (s, n + 1)
            div = _first_divergence(res["supports"][ii], res["k_used"][ii], gpu_sup[b], gpu_kused[b],
                                    scales, have, S, start)
            if div is None:
                final[b] = (res["coefs"][ii], res["k_used"][ii], res["xhat"][ii])
                continue
            s, n = div
            if n >= kstride or gpu_sup[b, s, n] < 0:
                rep.mismatched.append(b)          # the GPU stopped where the oracle went on
                continue
            forced[b, s, :n + 1] = gpu_sup[b, s, :n + 1]
            pending[b] = (s, n)
            nxt.append(b)
        active = np.array(nxt, dtype=np.int64)
    rep.mismatched.extend(int(b) for b in active)   # ran out of rounds
    for b, (coefs, ku, xh) in final.items():
        k = int(gpu_kused[b])
        if int(ku[S - 1]) != k:
            rep.k_used_diff += 1
            continue
        ref = coefs[S - 1, :k]
        den = np.linalg.norm(ref)
        if den > 0:
            rep.coef_rel_max = max(rep.coef_rel_max, float(np.linalg.norm(gpu_coef[b, :k] - ref) / den))
        if gpu_xhat is not None:
            xd = np.linalg.norm(xh)
            if xd > 0:
                rep.xhat_rel_max = max(rep.xhat_rel_max, float(np.linalg.norm(gpu_xhat[b] - xh) / xd))
    return rep


def _first_divergence(osup, oku, gsup, gku, scales, have, S, start=(0, 0)):
    for s in scales:
        if not have[s] or s < start[0]:
            continue
        ko = int(oku[s])
        kg = int(gku) if s == S - 1 else int(np.sum(gsup[s] >= 0))
        n0 = start[1] if s == start[0] else 0
        for n in range(n0, max(ko, kg)):
            a = osup[s, n] if n < ko else -1
            g = gsup[s, n] if n < kg else -1
            if a != g:
                return s, n
    return None


def _subset(w, idx):
    import synth
    return synth.subset(w, idx)
