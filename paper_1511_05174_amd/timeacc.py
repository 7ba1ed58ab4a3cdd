"""Time versus accuracy sweeps through the library, on synthetic signals.

The paper's evaluation method, at this library's speed:

  * dictionary size (Section II-C): full OMP (Algorithm 1) over single-scale
    dictionaries of T atoms at sparsity K -- time per patch against
    reconstruction PSNR, one curve per T as K grows;
  * time versus accuracy (Section IV, video denoising): the same
    single-scale points against zero-tree OMP (Algorithm 2) with K_low = 6
    and K_high = 8 over a two-scale dictionary of 512 / 8192 atoms, on
    8x8x32 video patches (coarse scale 4x4x16) at 15 dB input SNR;
  * the effect of Q = T_high / T_low (Section III-F, parameter selection):
    cross-scale dictionaries trained for several (T_low, Q) on one training
    set, denoising PSNR on held-out patches.

Signals come from the seeded generators of ``synth`` (the zero-tree model of
Section III with model dictionaries: children = the upsampled parent plus
detail), with white noise added here at the stated input SNR.  In the
video study the single-scale dictionary of T atoms is the model's fine
dictionary restricted to T of its atoms (a fixed random choice; T = 8192 is
all of it): the library's K-SVD update holds atoms of at most 64
coordinates, so dictionaries of 2048-coordinate atoms are not learned here.
The Q study learns its dictionaries (8x8 patches).  Everything runs on the
device through the C-ABI calls; this module only sequences them and times
them.
"""
from __future__ import annotations

import time
from typing import Optional, Sequence

import numpy as np

from . import cspd


def psnr_db(x: np.ndarray, xhat: np.ndarray) -> float:
    """10 log10(peak^2 / MSE) with peak = max |x| over the set."""
    mse = float(np.mean((xhat - x) ** 2))
    peak = float(np.max(np.abs(x)))
    return 10.0 * np.log10(peak * peak / max(mse, 1e-300))


def add_noise(x: np.ndarray, snr_db: float, rng: np.random.Generator) -> np.ndarray:
    """White Gaussian noise at the given input SNR (signal energy over noise
    energy, whole set)."""
    sig = float(np.mean(x * x))
    sigma = np.sqrt(sig / 10.0 ** (snr_db / 10.0))
    return x + sigma * rng.standard_normal(x.shape)


def _timed(fn, steps: int):
    """Seconds per call (mean over `steps` calls after one untimed call) and
    each kernel's mean duration in ms (the library's dispatch timestamps)."""
    torch = cspd._torch()
    fn()
    torch.cuda.synchronize()
    cspd.cspd_profile_reset()
    cspd.cspd_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    cspd.cspd_profile_enable(False)
    prof = {k: v[1] / max(v[0], 1) for k, v in cspd.cspd_profile_read().items()}
    return sec, prof


def _video_model(batch: int, seed: int, t_low: int, t_high: int, k_low: int, k_high: int):
    import synth

    grid, f = (32, 8, 8), (2, 2, 2)
    up, coarse = synth.box_map(grid, f)
    dims = [int(np.prod(coarse)), int(np.prod(grid))]
    w = synth.custom(dims, [t_low, t_high], batch, seed, k_scales=[k_low, k_high], sigma=0.0, up_maps=[up],
                     dict_kind="model", dtype="f32")
    return w, up


def video_time_accuracy(sizes: Sequence[int] = (256, 512, 1024, 4096, 8192), ks: Sequence[int] = (8, 16, 32, 64),
                        zt: tuple = (6, 8), t_low: int = 512, t_high: int = 8192, batch: int = 1024,
                        snr_db: float = 15.0, seed: int = 71, steps: int = 3) -> dict:
    """Single-scale full OMP over T atoms at each K, and zero-tree OMP at
    (K_low, K_high) = zt, on the same noisy 8x8x32 video patches.  Returns a
    dict with the points (ms per call, patches/s, PSNR) and, for every
    single-scale point, whether zero-tree OMP is at least as accurate and
    how much faster it is."""
    torch = cspd._torch()
    dev = torch.device("cuda", 0)
    w, up = _video_model(batch, seed, t_low, t_high, zt[0], zt[1])
    rng = np.random.default_rng(seed + 1)
    x = w.x
    y = add_noise(x, snr_db, rng)
    Y = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(dev)
    out = {"patches": batch, "shape": "8x8x32 video patches (2048 samples), coarse 4x4x16 (256)",
           "snr_in_db": snr_db, "psnr_noisy_db": psnr_db(x, y),
           "dictionaries": "model (single-scale: T atoms of the fine model dictionary)",
           "zero_tree": None, "single_scale": []}
    # zero-tree OMP over the two-scale model dictionary
    plan = cspd.cspd_plan(w.dims, w.atoms, w.dicts, w.up_maps, "identity", w.m, None, dtype="f32", k_max=16)
    res = {}

    def zt_call():
        res["r"] = cspd.cspd_omp_cross_scale(plan, Y, None, [zt[0]], None, zt[1])

    sec, prof = _timed(zt_call, steps)
    xh = res["r"][3].double().cpu().numpy()
    out["zero_tree"] = {"t_low": t_low, "t_high": t_high, "k_low": zt[0], "k_high": zt[1], "ms_per_call": sec * 1e3,
                        "patches_per_s": batch / sec, "psnr_db": psnr_db(x, xh), "kernels_ms": prof}
    cspd.cspd_plan_destroy(plan)
    # single-scale dictionaries
    perm = np.random.default_rng(seed + 2).permutation(t_high)
    kmax = max(ks)
    for T in sizes:
        d = w.dicts[1][np.sort(perm[:T])]
        plan = cspd.cspd_plan([w.n], [d.shape[0]], [d], [], "identity", w.n, None, dtype="f32", k_max=kmax)
        for K in ks:
            def full_call(K=K):
                res["r"] = cspd.cspd_omp_full(plan, Y, None, None, K)

            sec, prof = _timed(full_call, steps)
            xh = res["r"][3].double().cpu().numpy()
            pt = {"atoms": int(d.shape[0]), "k": int(K), "ms_per_call": sec * 1e3,
                  "patches_per_s": batch / sec, "psnr_db": psnr_db(x, xh), "kernels_ms": prof}
            # coefficient-coordinate kernel: its algorithmic bytes are the
            # Gram rows of the support, 4 T (1 + ... + K) per patch (the
            # FP64 correlations and Gram entries are smaller terms)
            kb = [v for k_, v in prof.items() if k_.startswith("omp_batch")]
            if kb:
                by = 4.0 * d.shape[0] * K * (K + 1) / 2 * batch
                pt["gram_bytes_per_call"] = by
                pt["gram_gb_per_s"] = by / (kb[0] * 1e-3) / 1e9
                pt["hbm_frac"] = pt["gram_gb_per_s"] / 8000.0
            out["single_scale"].append(pt)
        cspd.cspd_plan_destroy(plan)
    z = out["zero_tree"]
    for p in out["single_scale"]:
        p["zero_tree_psnr_gain_db"] = z["psnr_db"] - p["psnr_db"]
        p["zero_tree_speedup"] = p["ms_per_call"] / z["ms_per_call"]
    # the most accurate single-scale point, and the fastest one at least as
    # accurate as zero-tree OMP (within 0.1 dB), if any
    best = max(out["single_scale"], key=lambda p: p["psnr_db"])
    out["best_single_scale"] = best
    match = [p for p in out["single_scale"] if p["psnr_db"] >= z["psnr_db"] - 0.1]
    out["fastest_single_scale_within_0p1db"] = min(match, key=lambda p: p["ms_per_call"]) if match else None
    return out


def q_effect(t_lows: Sequence[int] = (64, 128), qs: Sequence[int] = (2, 4, 8, 16), k_low: int = 3,
             k_high: int = 4, train_patches: int = 16384, test_patches: int = 4096, snr_db: float = 15.0,
             iters_low: int = 4, iters_high: int = 4, seed: int = 81, truth: tuple = (128, 8)) -> dict:
    """Cross-scale dictionaries trained for each (T_low, Q) on the same
    training set of 8x8 patches (coarse 4x4) drawn from a two-scale model
    with T_low, Q = `truth`, and the denoising PSNR each gives on held-out
    patches at `snr_db` (zero-tree OMP at (k_low, k_high)).  The optimum
    reflects the generator; the method is the paper's cross-validation."""
    import synth

    from . import train

    torch = cspd._torch()
    dev = torch.device("cuda", 0)
    up, coarse = synth.box_map((8, 8), (2, 2))
    dims = [int(np.prod(coarse)), 64]
    tl0, q0 = truth
    w = synth.custom(dims, [tl0, tl0 * q0], train_patches + test_patches, seed, k_scales=[k_low, k_high],
                     sigma=0.0, up_maps=[up], dict_kind="model", dtype="f32")
    rng = np.random.default_rng(seed + 1)
    x = w.x
    y = add_noise(x, snr_db, rng)
    xtr, ytr = x[:train_patches], y[:train_patches]
    xte, yte = x[train_patches:], y[train_patches:]
    Yte = torch.from_numpy(np.ascontiguousarray(yte, dtype=np.float32)).to(dev)
    out = {"patches": "8x8 (coarse 4x4)", "truth": {"t_low": tl0, "q": q0}, "snr_in_db": snr_db,
           "train_patches": train_patches, "test_patches": test_patches, "k_low": k_low, "k_high": k_high,
           "points": []}
    for tl in t_lows:
        for q in qs:
            t0 = time.perf_counter()
            d_low, d_high = train.cross_scale(ytr, up, dims[0], tl, q, k_low, k_high, iters_low, iters_high,
                                              seed=seed + 2)
            t_train = time.perf_counter() - t0
            plan = cspd.cspd_plan(dims, [tl, tl * q], [d_low.astype(np.float64), d_high.astype(np.float64)],
                                  [up], "identity", 64, None, dtype="f32", k_max=16)
            r = cspd.cspd_omp_cross_scale(plan, Yte, None, [k_low], None, k_high)
            torch.cuda.synchronize()
            xh = r[3].double().cpu().numpy()
            out["points"].append({"t_low": tl, "q": q, "t_high": tl * q, "psnr_db": psnr_db(xte, xh),
                                  "train_s": t_train})
            cspd.cspd_plan_destroy(plan)
    for tl in t_lows:
        pts = [p for p in out["points"] if p["t_low"] == tl]
        out.setdefault("best_q", {})[str(tl)] = max(pts, key=lambda p: p["psnr_db"])["q"]
    return out


def main(argv: Optional[Sequence[str]] = None) -> int:
    import argparse
    import json

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--study", choices=["video", "q"], default="video")
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=3)
    args = ap.parse_args(argv)
    if args.study == "video":
        res = video_time_accuracy(batch=args.batch, steps=args.steps)
    else:
        res = q_effect()
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
