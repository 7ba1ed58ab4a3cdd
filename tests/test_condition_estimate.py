"""The condition estimate that decides where the FP32 kernels spend FP64
(CPU only).

The kernels estimate kappa(G) of the final support's Gram matrix as
tr(G) tr(G^-1) / n, accumulated while the support grows (tr(G) from the
pivots' squared norms, tr(G^-1) = ||L^-1||_F^2 from the columns of L^-1).
For symmetric positive definite G this lies between kappa(G) / n and
n kappa(G); the kernels refine the coefficients above 10 and re-solve them in
FP64 above 1e4 (one refinement step leaves about (kappa 2^-24)^2, which
reaches the 1e-5 tolerance near kappa ~ 5e4, hence the margin), and compute a
pivot in FP64 when the squared pivots' range exceeds 1e6.
"""
import numpy as np


def estimate(g):
    return np.trace(g) * np.trace(np.linalg.inv(g)) / g.shape[0]


def estimate_from_cholesky(g):
    """The kernel's route: tr(G) = sum of squared column norms (the pivots'
    e0), tr(G^-1) = ||L^-1||_F^2."""
    l = np.linalg.cholesky(g)
    li = np.linalg.inv(l)
    return np.trace(g) * np.sum(li * li) / g.shape[0]


def test_estimate_brackets_kappa():
    rng = np.random.default_rng(0)
    for n in range(2, 17):
        for _ in range(50):
            a = rng.standard_normal((max(n, 20), n))
            # stretch some directions to spread kappa over many decades
            a = a @ np.diag(10.0 ** rng.uniform(-4, 0, size=n))
            g = a.T @ a
            k = np.linalg.cond(g)
            e = estimate(g)
            assert k / n * (1 - 1e-9) <= e <= n * k * (1 + 1e-9)
            assert np.isclose(estimate_from_cholesky(g), e, rtol=1e-8)


def test_estimate_is_scale_free():
    """The kernels run on Gram matrices scaled by powers of two (the FP16
    split); the estimate and the pivot ratios must not move."""
    rng = np.random.default_rng(1)
    a = rng.standard_normal((32, 6))
    g = a.T @ a
    for s in (2.0 ** -20, 2.0 ** 14, 2.0 ** 28):
        assert np.isclose(estimate(s * g), estimate(g), rtol=1e-12)


def test_thresholds_reach_each_stage():
    """Two children that differ by delta on one sample: the deltas used by
    the GPU rescue tests land in the stages they name."""
    def pair(delta):
        a1 = np.ones(4)
        a2 = np.ones(4)
        a2[1] += delta
        g = np.stack([a1, a2], 1).T @ np.stack([a1, a2], 1)
        piv = g[1, 1] - g[0, 1] ** 2 / g[0, 0]
        return estimate(g), g[0, 0] / piv, piv / g[1, 1]

    e, ratio, rel = pair(2.0 ** -3)
    assert 10 < e < 1e4 and ratio < 1e6 and rel > 1e-5          # refinement only
    e, ratio, rel = pair(2.0 ** -7)
    assert e > 1e4 and ratio < 1e6 and rel > 1e-5               # FP64 re-solve
    e, ratio, rel = pair(2.0 ** -11)
    assert e > 1e4 and ratio > 1e6 and rel < 1e-5               # FP64 pivot and re-solve
    # and an orthonormal pair needs no FP64 at all
    # tr(G) tr(G^-1) >= n^2: the estimate of a perfectly conditioned support is n
    assert estimate(np.eye(2)) == 2.0 and estimate(np.eye(16)) == 16.0
