"""Compare a GPU run with the FP64 oracle, patch by patch.

Supports are compared step by step in selection order, at every scale.  At
the first step where they differ, the oracle is re-run with the GPU's picks
forced up to and including that step (its trace then holds, in FP64, the
score of its own best atom and of the GPU's pick).  The divergence is
excused as a near-tie when

    (best score - score of the GPU's pick) / (largest score at step 1 of
    that scale) < tie_tol

and the comparison continues against the replayed oracle; otherwise the
patch is a mismatch.  Excusals are counted and every caller bounds them.

Coefficients are compared entry by entry: each entry's error is measured
against the largest coefficient magnitude of that patch's oracle solution,
|a_gpu[i] - a_ref[i]| / max_j |a_ref[j]|, so a small coefficient cannot hide
inside a norm.  Reconstructions are compared norm-wise per patch.  Patches
that mismatch (or stop at another sparsity) are not dropped: they are listed,
with the scale, step and gap of the divergence, and their reconstruction is
compared with the oracle's own.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import oracle


@dataclass
class Report:
    patches: int
    mismatched: list = field(default_factory=list)     # patch ids with an unexcused divergence
    detail: dict = field(default_factory=dict)         # patch -> (scale, step, gap or reason)
    excused: int = 0                                   # near-ties excused
    k_used_diff: int = 0
    coef_rel_max: float = 0.0                          # max_i |d a_i| / ||a_ref||_inf
    coef_norm_rel_max: float = 0.0                     # ||d a||_2 / ||a_ref||_2
    xhat_rel_max: float = 0.0
    xhat_rel_max_mismatched: float = 0.0               # against the oracle's own x-hat
    worst_tie_gap: float = 0.0
    worst_coef_patch: int = -1

    def summary(self):
        return (f"patches={self.patches} mismatched={len(self.mismatched)} excused={self.excused} "
                f"coef_rel_max={self.coef_rel_max:.3e} (norm-wise {self.coef_norm_rel_max:.3e}) "
                f"xhat_rel_max={self.xhat_rel_max:.3e} worst_excused_gap={self.worst_tie_gap:.3e}"
                + (f" mismatched_xhat_rel_max={self.xhat_rel_max_mismatched:.3e}"
                   f" first={[(b, self.detail.get(b)) for b in self.mismatched[:4]]}"
                   if self.mismatched else ""))

    def check(self, coef_tol, xhat_tol, max_excused=None, max_mismatch=0):
        """Assert the parity bar.  max_excused defaults to 1 + patches // 500
        (0.2 %): FP32 rounding can only flip picks whose FP64 gap is below the
        near-tie tolerance, which random data makes rare."""
        if max_excused is None:
            max_excused = 1 + self.patches // 500
        assert len(self.mismatched) <= max_mismatch, self.summary()
        assert self.excused <= max_excused, f"excused {self.excused} > {max_excused}: {self.summary()}"
        assert self.k_used_diff == 0, self.summary()
        assert self.coef_rel_max <= coef_tol, self.summary()
        assert self.xhat_rel_max <= xhat_tol, self.summary()


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
    own_xhat = {}                     # the unforced oracle's x-hat (for mismatched patches)
    active = np.arange(B)

    def mismatch(b, why):
        rep.mismatched.append(b)
        rep.detail[b] = why

    for rnd in range(max_rounds + 1):
        if active.size == 0:
            break
        sub = _subset(w, active)
        res = oracle.omp(sub.dims, sub.atoms, sub.dicts, sub.up_maps, sub.phi_kind, sub.m, sub.phi,
                         sub.y, sub.mask, ks, k_fine=sub.k_fine, full=full, forced=forced[active],
                         kstride=kstride, with_trace=True, phase=getattr(sub, "phase", None))
        nxt = []
        for ii, b in enumerate(active):
            b = int(b)
            if rnd == 0:
                own_xhat[b] = res["xhat"][ii]
            start = (0, 0)
            if b in pending:
                s, n = pending.pop(b)
                if res["k_used"][ii, s] <= n:
                    mismatch(b, (s, n, "GPU pick not available to the oracle (chosen or dependent)"))
                    continue
                tr = res["trace"][ii, s, n]
                gap = (tr[0] - tr[2]) / tr[3] if tr[3] > 0 else np.inf
                if not gap < tie_tol:
                    mismatch(b, (s, n, float(gap)))
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
                mismatch(b, (s, n, "GPU stopped where the oracle went on"))
                continue
            forced[b, s, :n + 1] = gpu_sup[b, s, :n + 1]
            pending[b] = (s, n)
            nxt.append(b)
        active = np.array(nxt, dtype=np.int64)
    for b in active:
        mismatch(int(b), (-1, -1, "too many near-ties"))
    for b, (coefs, ku, xh) in final.items():
        k = int(gpu_kused[b])
        if int(ku[S - 1]) != k:
            rep.k_used_diff += 1
            rep.detail[b] = (S - 1, k, f"k_used {k} vs oracle {int(ku[S - 1])}")
            continue
        ref = coefs[S - 1, :k]
        amax = np.max(np.abs(ref)) if k else 0.0
        if amax > 0:
            d = np.abs(gpu_coef[b, :k] - ref)
            e = float(np.max(d) / amax)
            if e > rep.coef_rel_max:
                rep.coef_rel_max, rep.worst_coef_patch = e, b
            rep.coef_norm_rel_max = max(rep.coef_norm_rel_max, float(np.linalg.norm(d) / np.linalg.norm(ref)))
        elif k and np.any(gpu_coef[b, :k] != 0):
            rep.coef_rel_max = np.inf
        if gpu_xhat is not None:
            xd = np.linalg.norm(xh)
            if xd > 0:
                rep.xhat_rel_max = max(rep.xhat_rel_max, float(np.linalg.norm(gpu_xhat[b] - xh) / xd))
    if gpu_xhat is not None:
        for b in rep.mismatched:
            xh = own_xhat[b]
            xd = np.linalg.norm(xh)
            if xd > 0:
                rep.xhat_rel_max_mismatched = max(rep.xhat_rel_max_mismatched,
                                                  float(np.linalg.norm(gpu_xhat[b] - xh) / xd))
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
