"""Benchmark: batched zero-tree OMP on one MI355X.

One step is one cspd_omp_cross_scale call over the whole batch (every scale:
proxy, argmax, incremental Cholesky, projection, residue updates, output
and x-hat), with inputs already resident in device memory.  The default
workload is the 65,536-patch compressive inpainting set (8x8 patches, 4x4
coarse scale, D_high 64 x 1024, D_low 16 x 128, Q = 8, K = (4, 8), per-patch
50 % pixel masks, FP32).  The same batch is also solved with full OMP over
D_high for comparison, and the FP64 oracle is timed on the host cores.

Prints one JSON line.  --gpus above 1 is refused: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X, published FP32 vector rate
# The published FP32 vector rate counts packed FP32 (two FMAs per lane per
# instruction).  This library is built with packed FP32 off, so its vector
# code reaches at most half of it: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x
# 2.4 GHz = 78.6 TFLOP/s (the FP64 vector rate).  Reported beside the
# published peak, never in place of it.
PEAK_FP32_VECTOR_UNPACKED_TFLOPS = 78.6
PEAK_FP32_MATRIX_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def scale_flops(m: int, t_c: int, k: int, norms: bool) -> int:
    """Algorithmic FLOPs of K OMP iterations over t_c candidates of length m,
    with incremental least squares (the per-iteration cost model of the
    paper's Section III-D: proxy O(m t_c), argmax, least squares), plus the
    per-patch column norms when the operator differs per patch."""
    f = 0
    for n in range(1, k + 1):
        f += 2 * m * t_c + 2 * m * (n - 1) + (n - 1) ** 2 + 2 * m + 2 * n * n + 2 * m * n
    if norms:
        f += 2 * m * t_c
    return f


def kernel_flops(w, k_scales):
    """FLOPs per patch of each per-scale kernel of the cross-scale call and of
    the full-OMP call, keyed by the kernel role used in the profile labels.
    With a per-patch finest sparsity (w.k_fine) the finest scale's figure is
    the mean over the batch."""
    S = w.n_scales
    mask = w.phi_kind == "mask"
    out = {}
    kprev = None
    kf = None if w.k_fine is None else np.asarray(w.k_fine)
    for s in range(S):
        m = w.m if w.phi_kind == "dense" else w.dims[s]
        t_c = w.atoms[s] if s == 0 else min(w.atoms[s], (w.atoms[s] // w.atoms[s - 1]) * kprev)
        if s == S - 1 and kf is not None:
            vals, counts = np.unique(np.minimum(kf, t_c), return_counts=True)
            out[f"s{s}"] = float(sum(c * scale_flops(m, t_c, int(v), mask) for v, c in zip(vals, counts))
                                 / counts.sum())
            k = int(vals.max())
        else:
            k = min(k_scales[s], t_c)
            out[f"s{s}"] = scale_flops(m, t_c, k, mask)
        kprev = k
    m = w.m if w.phi_kind == "dense" else w.dims[-1]
    if kf is not None:
        vals, counts = np.unique(np.minimum(kf, w.atoms[-1]), return_counts=True)
        out["full"] = float(sum(c * scale_flops(m, w.atoms[-1], int(v), mask) for v, c in zip(vals, counts))
                            / counts.sum())
    else:
        out["full"] = scale_flops(m, w.atoms[-1], min(k_scales[-1], w.atoms[-1]), mask)
    return out


def bound_of(label: str) -> str:
    """Which roofline bounds a kernel, from its SQ counters: the full-search
    kernel and the batched correlation GEMM keep the matrix cores busy; the
    per-patch kernels (per-scale and first-scale) issue VALU on most cycles
    with the matrix cores under a quarter busy, so their bound is the vector
    ALU (priced against the FP32 vector peak)."""
    return "mfma" if label.startswith(("omp_full", "proxy_gemm")) else "alu"


def equal_psnr_phase(cspd, w, plan, timed):
    """The paper's time-accuracy method: full OMP at several K and zero-tree
    OMP over a (K_low, K_fine) grid on the same patches; for every full point
    the fastest zero-tree point whose PSNR is at least the full point's minus
    0.1 dB."""
    import torch
    B = w.batch
    dev = torch.device("cuda", 0)
    tdt = torch.float64 if w.dtype == "f64" else torch.float32
    ndt = np.float64 if w.dtype == "f64" else np.float32
    y = torch.from_numpy(np.ascontiguousarray(w.y.astype(ndt))).to(dev)
    mask = None if w.mask is None else torch.from_numpy(w.mask).to(dev)
    sup = torch.empty((B, plan.k_max), dtype=torch.int32, device=dev)
    coef = torch.empty((B, plan.k_max), dtype=tdt, device=dev)
    ku = torch.empty((B,), dtype=torch.int32, device=dev)
    xh = torch.empty((B, w.n), dtype=tdt, device=dev)
    stream = torch.cuda.current_stream()
    q = w.atoms[-1] // w.atoms[-2]
    full_pts = []
    for kf_ in (2, 3, 4, 5, 6, 8):
        if kf_ > plan.k_max:
            continue

        def step_f(k=kf_):
            cspd.cspd_omp_full(plan, y, mask, None, k, support=sup, coef=coef, k_used=ku, xhat=xh,
                               stream=stream)
        t_f, _ = timed(step_f, 3, 1)
        full_pts.append({"k": kf_, "psnr_db": psnr_db(w.x, xh.double().cpu().numpy()),
                         "patches_per_s": B / t_f})
    cross_pts = []
    for k_low in (2, 3, 4, 6, 8):
        for k_fine in (3, 4, 5, 6, 8, 10, 12):
            if k_fine > min(q * k_low, plan.k_max) or q * k_low > 128:
                continue
            kk = [k_low, k_fine]

            def step_k(kk=kk):
                cspd.cspd_omp_cross_scale(plan, y, mask, kk[:-1], None, kk[-1], support=sup, coef=coef,
                                          k_used=ku, xhat=xh, stream=stream)
            try:
                t_k, _ = timed(step_k, 5, 1)
            except cspd.CspdError:
                continue
            cross_pts.append({"k_low": k_low, "k_fine": k_fine,
                              "psnr_db": psnr_db(w.x, xh.double().cpu().numpy()),
                              "patches_per_s": B / t_k})
    pairs = []
    for fp in full_pts:
        ok = [c for c in cross_pts if c["psnr_db"] >= fp["psnr_db"] - 0.1]
        best = max(ok, key=lambda c: c["patches_per_s"]) if ok else None
        pairs.append({"full": fp, "cross": best,
                      "speedup": None if best is None else best["patches_per_s"] / fp["patches_per_s"]})
    matched = [p for p in pairs if p["cross"] is not None]
    head = max(matched, key=lambda p: p["full"]["psnr_db"]) if matched else None
    best_full = max(full_pts, key=lambda p: p["psnr_db"]) if full_pts else None
    best_cross = max(cross_pts, key=lambda p: p["psnr_db"]) if cross_pts else None
    equal = {"child_detail": w.meta.get("child_detail"), "pairs": pairs,
             "best_matched_full_k": None if head is None else head["full"]["k"],
             "speedup_at_best_matched": None if head is None else head["speedup"],
             "best_psnr_db_full": None if best_full is None else best_full["psnr_db"],
             "best_psnr_db_cross": None if best_cross is None else best_cross["psnr_db"],
             "full_sweep": full_pts, "cross_sweep": cross_pts}
    for p in pairs:
        print(f"[bench] detail {w.meta.get('child_detail')}: full K={p['full']['k']} psnr "
              f"{p['full']['psnr_db']:.2f} dB {p['full']['patches_per_s']:.3e}/s -> cross {p['cross']} "
              f"speedup {p['speedup']}", file=sys.stderr, flush=True)
    return equal


def workloads_phase(cspd, names=("c1", "c3", "c4", "c4loc", "bayer", "lfca"), steps: int = 10, warmup: int = 2):
    """The other configurations at their full sizes, same timing as the
    headline (inputs resident, one cross-scale call per step, per-kernel
    durations from the dispatches' own timestamps); the structured-operator
    workloads (location-dependent coded exposure through the per-patch
    operator call, Bayer demosaicing, coded-aperture light fields) too."""
    import torch
    import synth
    res = {}
    for name in names:
        w = synth.make(name)
        B = w.batch
        ks = list(w.k_scales)
        plan = cspd.plan_from_workload(w)
        tdt = torch.float64 if w.dtype == "f64" else torch.float32
        ndt = np.float64 if w.dtype == "f64" else np.float32
        dev = torch.device("cuda", 0)
        y = torch.from_numpy(np.ascontiguousarray(w.y.astype(ndt))).to(dev)
        mask = None if w.mask is None else torch.from_numpy(w.mask).to(dev)
        kf = None if w.k_fine is None else torch.from_numpy(w.k_fine.astype(np.int32)).to(dev)
        sup = torch.empty((B, plan.k_max), dtype=torch.int32, device=dev)
        coef = torch.empty((B, plan.k_max), dtype=tdt, device=dev)
        ku = torch.empty((B,), dtype=torch.int32, device=dev)
        xh = torch.empty((B, w.n), dtype=tdt, device=dev)
        stream = torch.cuda.current_stream()
        ph = None if w.phase is None else torch.from_numpy(np.ascontiguousarray(w.phase, dtype=np.int32)).to(dev)

        def step():
            if ph is not None:
                cspd.cspd_omp_cross_scale_phased(plan, ph, y, mask, ks[:-1], kf, ks[-1], support=sup, coef=coef,
                                                 k_used=ku, xhat=xh, stream=stream)
            else:
                cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1], support=sup, coef=coef,
                                          k_used=ku, xhat=xh, stream=stream)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        cspd.cspd_profile_reset()
        cspd.cspd_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        cspd.cspd_profile_enable(False)
        prof = cspd.cspd_profile_read()
        flops = kernel_flops(w, ks)
        label, (launches, tot_ms) = max(prof.items(), key=lambda kv: kv[1][1])
        role = label.split(":")[-1]
        avg_ms = tot_ms / max(launches, 1)
        per_patch = flops.get(role)
        achieved = per_patch * B / (avg_ms * 1e-3) / 1e12 if per_patch else None
        peak = PEAK_FP32_VECTOR_TFLOPS if w.dtype == "f32" else PEAK_FP64_VECTOR_TFLOPS
        res[name] = {
            "workload": f"{name}: {B} patches, dims {w.dims}, atoms {w.atoms}, K {ks}"
                        + (" (finest K per patch)" if w.k_fine is not None else "")
                        + f", phi {w.phi_kind}"
                        + (f" ({int(np.max(w.phase)) + 1} operators chosen per patch)" if w.phase is not None else "")
                        + f", {w.dtype}",
            "patches_per_s": B / t, "ms_per_call": t * 1e3, "dtype": w.dtype,
            "roofline": {"bound": bound_of(label), "achieved": achieved, "peak": peak,
                         "unit": "TFLOP/s", "frac": None if achieved is None else achieved / peak,
                         "traffic": None, "kernel": label, "kernel_ms": avg_ms, "flops_per_patch": per_patch},
            "kernels": {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)} for k, v in prof.items()},
        }
        print(f"[bench] {name}: {B / t / 1e6:.1f} M patches/s, {t * 1e3:.3f} ms/call, dominant {label} "
              f"{avg_ms:.3f} ms", file=sys.stderr, flush=True)
        del y, mask, kf, sup, coef, ku, xh, plan, ph
        torch.cuda.synchronize()
    return res


COPY_PROBE_FLOATS = 64 << 20   # 256 MiB read and written by the calibration pass


def kernel_source_hash():
    """Hash of the sources of the cross-scale kernels (the first-scale and
    per-scale kernels and what they include); a traffic summary taken on other
    sources is not used."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1511_05174_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.startswith(("omp_scale", "omp_first", "proxy_gemm", "cspd_internal")) and name.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, name), "rb").read())
    # per-file compiler flags change the kernels too
    h.update(open(os.path.join(ROOT, "paper_1511_05174_amd", "build.py"), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel_role: str, launches_per_step: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    ent = d.get("kernels", {}).get(kernel_role)
    return None if ent is None else ent.get("hbm_bytes_per_launch")


def psnr_db(x, xhat):
    err = np.mean((x - xhat) ** 2)
    peak = np.max(np.abs(x))
    return float(10 * np.log10(peak * peak / err))


def snr_db(x, xhat):
    return float(20 * np.log10(np.linalg.norm(x) / np.linalg.norm(x - xhat)))


SERVE_SHAPES = ("c5a", "c5b", "c5c")


def serve_phase(cspd, jobs=2000, loads=(0.5, 0.8, 0.95), budget=4 << 30, slots=4, pool=32768,
                bmax=262144, burst=150, ring=8, seed=11):
    """Serving on the three job shapes (64-d image, 512-d video, 400-d light
    field; Gaussian Phi at 25 %, K_low 4): job sizes log-uniform integers in
    [1024, bmax] patches, shape uniform, each job's K_fine uniform in 6..16.
    Capacity = patches/s of a burst of `burst` jobs submitted at once; then
    `jobs` Poisson arrivals at each offered load (fraction of capacity).
    Inputs and outputs are pinned host buffers allocated up front (outputs:
    a ring of `ring` job-sized sets, so at most `ring` jobs are outstanding;
    the client waits for the oldest when all are taken); latency = finish -
    submit as the server records it (queueing, admission, PCIe both ways,
    kernels).  The same burst is also run on device-resident jobs (inputs in
    HBM, outputs written in place) for the capacity without PCIe."""
    import torch

    import synth

    rng = np.random.default_rng(seed)
    shapes = {}
    for name in SERVE_SHAPES:
        w = synth.make(name, batch=pool)
        plan = cspd.plan_from_workload(w)
        y = torch.empty((bmax, w.m), dtype=torch.float32, pin_memory=True).numpy()
        y[:] = np.tile(w.y.astype(np.float32), (bmax // pool, 1))
        shapes[name] = (w, plan, y)

    def draw(n):
        size = np.floor(np.exp(rng.uniform(np.log(1024), np.log(bmax + 1), size=n))).astype(np.int64)
        size = np.clip(size, 1024, bmax)
        return dict(shape=rng.integers(0, len(SERVE_SHAPES), size=n), size=size,
                    start=np.array([rng.integers(0, bmax - b + 1) for b in size]),
                    k=rng.integers(6, 17, size=n))

    kmax = max(shapes[nm][1].k_max for nm in SERVE_SHAPES)
    nmax = max(shapes[nm][1].n for nm in SERVE_SHAPES)

    def pinned(count, dt):
        return torch.empty(count, dtype=dt, pin_memory=True).numpy()

    free_sets = [{"support": pinned(bmax * kmax, torch.int32), "k_used": pinned(bmax, torch.int32),
                  "coef": pinned(bmax * kmax, torch.float32), "xhat": pinned(bmax * nmax, torch.float32)}
                 for _ in range(ring)]

    def collect(srv, held, rows, block, oldest_only=False):
        for jid in sorted(held)[:1] if oldest_only else list(held):
            r = cspd.cspd_serve_poll(srv, jid, -1 if block else 0)
            if r is None:
                continue
            _, st = r
            name, n, bufs = held.pop(jid)
            free_sets.append(bufs)
            rows.append((name, n, (st["finish_ns"] - st["submit_ns"]) * 1e-6,
                         (st["admit_ns"] - st["submit_ns"]) * 1e-6, st["batched_with"] > 0))

    def submit(srv, d, i, held, rows):
        name = SERVE_SHAPES[int(d["shape"][i])]
        w, plan, y = shapes[name]
        n, a = int(d["size"][i]), int(d["start"][i])
        while not free_sets:
            collect(srv, held, rows, True, oldest_only=True)
        bufs = free_sets.pop()
        out = {"support": bufs["support"][:n * plan.k_max].reshape(n, plan.k_max), "k_used": bufs["k_used"][:n],
               "coef": bufs["coef"][:n * plan.k_max].reshape(n, plan.k_max),
               "xhat": bufs["xhat"][:n * plan.n].reshape(n, plan.n)}
        jid = cspd.cspd_serve_submit(srv, plan, y[a:a + n], None, None, int(d["k"][i]), w.k_scales[:-1], out=out)
        held[jid] = (name, n, bufs)
        return jid

    srv = cspd.cspd_serve_create(0, budget, slots)
    # warm-up: a small job per shape and sparsity bucket (loads every kernel
    # the measured jobs use)
    held, rows = {}, []
    for si in range(len(SERVE_SHAPES)):
        for kk in (6, 16):
            submit(srv, dict(shape=[si], size=[4096], start=[0], k=[kk]), 0, held, rows)
            collect(srv, held, rows, True)
    d = draw(burst)
    rows = []
    t0 = time.perf_counter()
    for i in range(burst):
        submit(srv, d, i, held, rows)
    collect(srv, held, rows, True)
    cap = float(d["size"].sum()) / (time.perf_counter() - t0)
    # the same burst with device-resident jobs: inputs already in HBM, outputs
    # written in place (no PCIe); a ring of `ring` device output sets
    dev = torch.device("cuda", 0)
    dev_y = {nm: torch.from_numpy(shapes[nm][2]).to(dev) for nm in SERVE_SHAPES}
    dev_sets = [{"support": torch.empty(bmax * kmax, dtype=torch.int32, device=dev),
                 "k_used": torch.empty(bmax, dtype=torch.int32, device=dev),
                 "coef": torch.empty(bmax * kmax, dtype=torch.float32, device=dev),
                 "xhat": torch.empty(bmax * nmax, dtype=torch.float32, device=dev)} for _ in range(ring)]
    dheld = []

    def dev_submit(i):
        name = SERVE_SHAPES[int(d["shape"][i])]
        w, plan, _ = shapes[name]
        n, a = int(d["size"][i]), int(d["start"][i])
        if not dev_sets:
            jid, bufs = dheld.pop(0)
            cspd.cspd_serve_poll(srv, jid, -1)
            dev_sets.append(bufs)
        bufs = dev_sets.pop()
        jid = cspd.cspd_serve_submit_device(
            srv, plan, dev_y[name][a:a + n], None, None, int(d["k"][i]), w.k_scales[:-1],
            support=bufs["support"][:n * plan.k_max].view(n, plan.k_max), coef=bufs["coef"][:n * plan.k_max].view(
                n, plan.k_max), k_used=bufs["k_used"][:n], xhat=bufs["xhat"][:n * plan.n].view(n, plan.n))
        dheld.append((jid, bufs))

    for i in range(min(6, burst)):      # warm-up of the in-place path
        dev_submit(i)
    while dheld:
        jid, bufs = dheld.pop(0)
        cspd.cspd_serve_poll(srv, jid, -1)
        dev_sets.append(bufs)
    t0 = time.perf_counter()
    for i in range(burst):
        dev_submit(i)
    while dheld:
        jid, bufs = dheld.pop(0)
        cspd.cspd_serve_poll(srv, jid, -1)
        dev_sets.append(bufs)
    cap_dev = float(d["size"].sum()) / (time.perf_counter() - t0)
    del dev_y, dev_sets
    mean_size = (bmax + 1 - 1024) / np.log((bmax + 1) / 1024.0)
    out = {"shapes": {n: f"{shapes[n][0].dims} atoms {shapes[n][0].atoms} M {shapes[n][0].m}"
                      for n in SERVE_SHAPES},
           "job_patches": f"log-uniform integer in [1024, {bmax}]", "k_fine": "uniform 6..16 per job",
           "capacity_patches_per_s": cap, "capacity_device_buffers_patches_per_s": cap_dev,
           "capacity_burst_jobs": burst, "slots": slots,
           "client_ring": ring,
           "hbm_budget_bytes": budget, "jobs_per_load": jobs, "loads": {}}
    for load in loads:
        d = draw(jobs)
        rate = load * cap / mean_size
        gaps = rng.exponential(1.0 / rate, size=jobs)
        rows = []
        t_start = time.perf_counter()
        t_next = t_start
        for i in range(jobs):
            t_next += gaps[i]
            # between arrivals: retire finished jobs (the oldest first), then
            # sleep briefly rather than spin on the server's lock
            while True:
                now = time.perf_counter()
                if now >= t_next:
                    break
                if held:
                    collect(srv, held, rows, False, oldest_only=True)
                time.sleep(min(t_next - now, 2e-4))
            submit(srv, d, i, held, rows)
        collect(srv, held, rows, True)
        wall = time.perf_counter() - t_start
        lat = np.array([r[2] for r in rows])
        adm = np.array([r[3] for r in rows])
        ent = {"rate_jobs_per_s": rate, "wall_s": wall, "patches_per_s": float(d["size"].sum()) / wall,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "mean_ms": float(lat.mean()), "admission_wait_p99_ms": float(np.percentile(adm, 99)),
               "batched_jobs": int(sum(r[4] for r in rows)), "per_shape": {}}
        for name in SERVE_SHAPES:
            ls = np.array([r[2] for r in rows if r[0] == name])
            if len(ls):
                ent["per_shape"][name] = {"jobs": int(len(ls)), "p50_ms": float(np.percentile(ls, 50)),
                                          "p99_ms": float(np.percentile(ls, 99))}
        small = np.array([r[2] for r in rows if r[1] <= 8192])
        if len(small):
            ent["small_jobs_le_8192"] = {"jobs": int(len(small)), "p50_ms": float(np.percentile(small, 50)),
                                         "p99_ms": float(np.percentile(small, 99))}
        out["loads"][str(load)] = ent
        print(f"[bench] serving load {load}: {json.dumps(ent)}", file=sys.stderr, flush=True)
    cspd.cspd_serve_destroy(srv)
    for name in SERVE_SHAPES:
        cspd.cspd_plan_destroy(shapes[name][1])
    return out


def precision_phase(cspd, steps: int = 3):
    """Reduced-precision proxy study on the three-scale workload (262,144
    patches): full OMP over its finest scale (4096 atoms of length 128, K =
    12) and cross-scale OMP over all three scales, each with the FP32 proxy
    and with bf16 / fp16 proxies plus FP32 re-scoring: time per call and how
    far each result is from the FP32 path's.  (Errors against the FP64
    oracle come from the parity tests, which run the oracle.)"""
    import torch

    import synth

    w = synth.make("c3")
    B = w.batch
    K = w.k_scales[-1]
    dev = torch.device("cuda", 0)
    y = torch.from_numpy(np.ascontiguousarray(w.y.astype(np.float32))).to(dev)
    out = {"workload": f"c3 finest scale: {B} patches, {w.atoms[-1]} atoms of length {w.m}, K {K}",
           "modes": {}}
    ref = None
    for mode in ("native", "bf16", "f16"):
        plan = cspd.plan_from_workload(w, corr_mode=mode)
        sup, coef, ku, xh = cspd.cspd_omp_full(plan, y, None, None, K)
        torch.cuda.synchronize()
        cspd.cspd_profile_reset()
        cspd.cspd_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            cspd.cspd_omp_full(plan, y, None, None, K, support=sup, coef=coef, k_used=ku, xhat=xh)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cspd.cspd_profile_enable(False)
        prof = cspd.cspd_profile_read()
        s_np = sup.cpu().numpy()
        x_np = xh.double().cpu().numpy()
        ent = {"ms_per_call": (t1 - t0) / steps * 1e3, "patches_per_s": B * steps / (t1 - t0),
               "kernels": {k: v[1] / max(v[0], 1) for k, v in prof.items()}}
        if ref is None:
            ref = (s_np, x_np)
        else:
            d = np.linalg.norm(x_np - ref[1], axis=1) / np.maximum(np.linalg.norm(ref[1], axis=1), 1e-30)
            ent["same_support_as_fp32"] = float(np.mean(np.all(s_np == ref[0], axis=1)))
            ent["xhat_rel_diff_vs_fp32_q99"] = float(np.quantile(d, 0.99))
            ent["xhat_rel_diff_vs_fp32_max"] = float(d.max())
            ent["speedup_vs_fp32"] = out["modes"]["native"]["ms_per_call"] / ent["ms_per_call"]
        out["modes"][mode] = ent
        cspd.cspd_plan_destroy(plan)
    # cross-scale OMP on the same workload: scale 0's correlations with y from
    # the FP32 / bf16 / fp16 batched contraction, FP32 re-scoring before each
    # first-scale pick
    ks = w.k_scales
    out["cross"] = {"workload": f"c3 cross-scale: {B} patches, dims {w.dims}, atoms {w.atoms}, K {ks}",
                    "modes": {}}
    ref = None
    for mode in ("native", "bf16", "f16"):
        plan = cspd.plan_from_workload(w, corr_mode=mode)
        res = cspd.cspd_omp_cross_scale(plan, y, None, ks[:-1], None, ks[-1])
        torch.cuda.synchronize()
        cspd.cspd_profile_reset()
        cspd.cspd_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            cspd.cspd_omp_cross_scale(plan, y, None, ks[:-1], None, ks[-1], support=res[0], coef=res[1],
                                      k_used=res[2], xhat=res[3])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cspd.cspd_profile_enable(False)
        prof = cspd.cspd_profile_read()
        s_np = res[0].cpu().numpy()
        x_np = res[3].double().cpu().numpy()
        ent = {"ms_per_call": (t1 - t0) / steps * 1e3, "patches_per_s": B * steps / (t1 - t0),
               "kernels": {k: v[1] / max(v[0], 1) for k, v in prof.items()}}
        if ref is None:
            ref = (s_np, x_np)
        else:
            d = np.linalg.norm(x_np - ref[1], axis=1) / np.maximum(np.linalg.norm(ref[1], axis=1), 1e-30)
            ent["same_support_as_fp32"] = float(np.mean(np.all(s_np == ref[0], axis=1)))
            ent["xhat_rel_diff_vs_fp32_q99"] = float(np.quantile(d, 0.99))
            ent["xhat_rel_diff_vs_fp32_max"] = float(d.max())
            ent["speedup_vs_fp32"] = out["cross"]["modes"]["native"]["ms_per_call"] / ent["ms_per_call"]
        out["cross"]["modes"][mode] = ent
        cspd.cspd_plan_destroy(plan)
    return out


def graph_phase(cspd, w, ks, sizes=(1024, 8192, 65536), reps=50):
    """Wall time per call of a cross-scale call issued eagerly (library call
    per batch: workspace, one launch per scale) and replayed from a captured
    HIP graph, at several batch sizes (slices of the workload)."""
    import torch

    import synth

    plan = cspd.plan_from_workload(w)
    out = {}
    for n in sizes:
        n = min(n, w.batch)
        sub = synth.subset(w, np.arange(n))
        ndt = np.float64 if w.dtype == "f64" else np.float32
        y = torch.from_numpy(np.ascontiguousarray(sub.y.astype(ndt))).cuda()
        mask = None if sub.mask is None else torch.from_numpy(np.ascontiguousarray(sub.mask)).cuda()
        res = cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], None, ks[-1])
        g, *_ = cspd.cspd_graph_cross_scale(plan, y, mask, ks[:-1], None, ks[-1])

        def eager():
            cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], None, ks[-1], support=res[0], coef=res[1],
                                      k_used=res[2], xhat=res[3])

        def replay():
            cspd.cspd_graph_launch(g)

        ent = {}
        for name, fn in (("eager", eager), ("graph", replay)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            ent[f"{name}_us"] = (time.perf_counter() - t0) / reps * 1e6
        ent["graph_speedup"] = ent["eager_us"] / ent["graph_us"]
        out[str(n)] = ent
        del g
    return out


def autotune_phase(cspd, w, ks, y, mask, kf, steps: int = 10):
    """Autotuner on the benchmark batch: the kernel it keeps per scale, and the
    time per cross-scale step with the tuned plan against the shape rules
    (two plans of the same workload, timed alternately)."""
    import torch

    rules = cspd.plan_from_workload(w)
    tuned = cspd.plan_from_workload(w)
    t0 = time.perf_counter()
    cspd.cspd_autotune(tuned, y, mask, ks[:-1], kf, ks[-1], reps=3)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    chosen = {}
    for s in range(w.n_scales):
        kb = 0 if ks[s] <= 4 else (1 if ks[s] <= 8 else 2)
        kind, nc, ppw, cand = cspd.cspd_tuned_kernel(tuned, s, kb)
        chosen[f"s{s}"] = {"kind": kind, "nc": nc, "ppw": ppw, "cand": cand}
    res = {}
    for name, plan in (("rules", rules), ("tuned", tuned)):
        out = cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1], support=out[0], coef=out[1],
                                      k_used=out[2], xhat=out[3])
        torch.cuda.synchronize()
        res[f"{name}_ms"] = (time.perf_counter() - t0) / steps * 1e3
    res["speedup"] = res["rules_ms"] / res["tuned_ms"]
    res["tune_s"] = tune_s
    res["chosen"] = chosen
    return res


def pipeline_phase(cspd, w, ks, reps: int = 5):
    """Whole-image inpainting: the workload's 65,536 patches tiled into a
    2048 x 2048 image, half of its pixels kept (Bernoulli 1/2), then cut into
    overlapping 8 x 8 patches at stride 4 (261,121 patches), zero-tree OMP
    (and full OMP for comparison) on the inpainting plan, and averaging.
    Times per stage on the device (events), image PSNR against the clean
    image."""
    import torch

    side, tile = 2048, 8
    per = side // tile
    clean = w.x.reshape(per, per, tile, tile).transpose(0, 2, 1, 3).reshape(side, side).astype(np.float32)
    rng = np.random.default_rng(21)
    mask = (rng.random((side, side)) < 0.5).astype(np.uint8)
    meas = (clean * mask).astype(np.float32)
    grid = cspd.patch_grid((side, side), (tile, tile), (4, 4))
    n = cspd.cspd_patch_count(grid)
    plan = cspd.plan_from_workload(w)
    dev = torch.device("cuda", 0)
    m_t = torch.from_numpy(mask).to(dev)
    s_t = torch.from_numpy(meas).to(dev)
    y, pm = cspd.cspd_extract_patches(grid, s_t, m_t)
    out = cspd.cspd_omp_cross_scale(plan, y, pm, ks[:-1], None, ks[-1])
    img = cspd.cspd_aggregate_patches(grid, out[3])
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    times = {"extract_ms": 0.0, "omp_ms": 0.0, "aggregate_ms": 0.0}
    for _ in range(reps):
        ev[0].record()
        cspd.cspd_extract_patches(grid, s_t, m_t, y=y, patch_mask=pm)
        ev[1].record()
        cspd.cspd_omp_cross_scale(plan, y, pm, ks[:-1], None, ks[-1], support=out[0], coef=out[1], k_used=out[2],
                                  xhat=out[3])
        ev[2].record()
        cspd.cspd_aggregate_patches(grid, out[3], out=img)
        ev[3].record()
        torch.cuda.synchronize()
        times["extract_ms"] += ev[0].elapsed_time(ev[1]) / reps
        times["omp_ms"] += ev[1].elapsed_time(ev[2]) / reps
        times["aggregate_ms"] += ev[2].elapsed_time(ev[3]) / reps
    img_cross = img.cpu().numpy()
    fo = cspd.cspd_omp_full(plan, y, pm, None, ks[-1])
    fimg = cspd.cspd_aggregate_patches(grid, fo[3])
    torch.cuda.synchronize()
    ev[0].record()
    cspd.cspd_omp_full(plan, y, pm, None, ks[-1], support=fo[0], coef=fo[1], k_used=fo[2], xhat=fo[3])
    ev[1].record()
    torch.cuda.synchronize()
    full_ms = ev[0].elapsed_time(ev[1])
    img_full = fimg.cpu().numpy()
    total = sum(times.values())
    res = {"image": f"{side} x {side}, 8x8 patches at stride 4, half of the pixels observed",
           "patches": n, **{k: round(v, 4) for k, v in times.items()}, "total_ms": round(total, 4),
           "megapixels_per_s": side * side / (total * 1e-3) / 1e6,
           "psnr_db_cross": psnr_db(clean.astype(np.float64), img_cross.astype(np.float64)),
           "psnr_db_full": psnr_db(clean.astype(np.float64), img_full.astype(np.float64)),
           "full_omp_ms": round(full_ms, 4), "omp_speedup_vs_full": full_ms / times["omp_ms"]}
    cspd.cspd_plan_destroy(plan)
    return res


def learning_phase(cspd, w, iters: int = 3):
    """Section III-E on the workload's 65,536 clean patches: cross-scale
    learning (K-SVD on the down-sampled set for D_low, then K-SVD with
    zero-tree OMP for D_high: T 128 / 1024, K 4 / 8) against plain K-SVD of a
    1024-atom dictionary with full OMP (K 8).  Per-iteration time of the
    sparse-approximation step and of the dictionary update, and the relative
    representation error ||X - D S|| / ||X|| after the last iteration."""
    import torch

    from paper_1511_05174_amd import train

    x = w.x.astype(np.float64)
    n_low, t_low, q = w.dims[0], w.atoms[0], w.atoms[1] // w.atoms[0]
    k_low, k_high = w.k_scales
    tm = {}
    d_low, d_high = train.cross_scale(x, w.up_maps[0], n_low, t_low, q, k_low, k_high, iters, iters, seed=5,
                                      timings=tm)
    rng = np.random.default_rng(6)
    d0 = train._unit_rows(x[rng.choice(len(x), size=w.atoms[1], replace=False)])
    tp = []
    d_plain, sup_p, coef_p = train.ksvd(x, d0, k_high, iters, tp)

    def rel_err(D, sup, coef):
        rec = np.zeros_like(x)
        for j in range(sup.shape[1]):
            a = sup[:, j]
            ok = a >= 0
            rec[ok] += coef[ok, j:j + 1] * D[a[ok]]
        return float(np.linalg.norm(x - rec) / np.linalg.norm(x))

    # representation error of the learned pair: one more zero-tree coding
    plan = train._plan([n_low, w.dims[1]], [t_low, t_low * q], [d_low.astype(np.float64), d_high.astype(np.float64)],
                       [w.up_maps[0]], max(k_low, k_high))
    X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    sup_c, coef_c, _, _ = cspd.cspd_omp_cross_scale(plan, X, None, [k_low], None, k_high, want_xhat=False)
    err_cross = rel_err(d_high.astype(np.float64), sup_c.cpu().numpy(), coef_c.cpu().numpy().astype(np.float64))
    cspd.cspd_plan_destroy(plan)
    err_plain = rel_err(d_plain.astype(np.float64), sup_p, coef_p.astype(np.float64))
    hi = np.array(tm["high"])
    pl = np.array(tp)
    return {"signals": int(len(x)), "iterations": iters,
            "cross_scale": {"coding_ms": float(hi[:, 0].mean() * 1e3), "update_ms": float(hi[:, 1].mean() * 1e3),
                            "step1_iter_ms": float(np.array(tm["low"]).sum(axis=1).mean() * 1e3),
                            "rel_error": err_cross},
            "plain_ksvd": {"coding_ms": float(pl[:, 0].mean() * 1e3), "update_ms": float(pl[:, 1].mean() * 1e3),
                           "rel_error": err_plain},
            "coding_speedup": float(pl[:, 0].mean() / hi[:, 0].mean()),
            "iteration_speedup": float(pl.sum(axis=1).mean() / hi.sum(axis=1).mean())}


def traffic_probe(workload: str, steps: int = 3):
    """A plain elementwise pass over a buffer of known size, then a few
    cross-scale steps: run under rocprofv3 --pmc FETCH_SIZE, and again under
    WRITE_SIZE, then summarize both with --traffic-summarize."""
    import torch

    import synth
    from paper_1511_05174_amd import cspd

    dev = torch.device("cuda", 0)
    n = COPY_PROBE_FLOATS
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)      # reads 4 n bytes, writes 4 n bytes
    torch.cuda.synchronize()
    w = synth.make(workload)
    ks = list(w.k_scales)
    plan = cspd.plan_from_workload(w)
    ndt = np.float64 if w.dtype == "f64" else np.float32
    y = torch.from_numpy(np.ascontiguousarray(w.y.astype(ndt))).to(dev)
    mask = None if w.mask is None else torch.from_numpy(w.mask).to(dev)
    kf = None if w.k_fine is None else torch.from_numpy(w.k_fine.astype(np.int32)).to(dev)
    for _ in range(steps):
        cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1])
    torch.cuda.synchronize()
    print(json.dumps({"probe": workload, "copy_floats": n, "steps": steps, "scales": w.n_scales}))


def traffic_summarize(fetch_db: str, write_db: str, workload: str, command: str):
    """HBM bytes per launch of each scale's kernel from the two counter runs
    of --traffic-probe, each counter scaled by what it reads for the plain
    elementwise pass (4 n bytes fetched and 4 n written)."""
    import sqlite3

    import synth

    def dispatches(db, counter):
        c = sqlite3.connect(db)
        rows = c.execute("select dispatch_id, kernel_name, sum(value) from counters_collection "
                         "where counter_name = ? group by dispatch_id order by dispatch_id",
                         (counter,)).fetchall()
        return [(k, float(v)) for _, k, v in rows]

    s_count = synth.make(workload, batch=1).n_scales
    out = {"workload": workload, "source_hash": kernel_source_hash(), "command": command,
           "copy_bytes_each_way": 4 * COPY_PROBE_FLOATS, "kernels": {}}
    for counter, key in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        rows = dispatches(fetch_db if key == "fetch" else write_db, counter)
        copies = [v for k, v in rows if "elementwise" in k]
        omp = [(k, v) for k, v in rows if "k_omp_" in k]
        copy_kib = float(np.median(copies))
        factor = 4 * COPY_PROBE_FLOATS / (copy_kib * 1024.0)
        out[f"{key}_factor"] = factor
        out[f"copy_{key}_kib"] = copy_kib
        for i, (k, v) in enumerate(omp):
            role = f"s{i % s_count}" if s_count > 1 else "full"
            ent = out["kernels"].setdefault(role, {"name": k.split("(")[0], f"{key}_kib": []})
            ent.setdefault(f"{key}_kib", []).append(v)
            out[f"{key}_factor"] = factor
    for role, ent in out["kernels"].items():
        fk = float(np.median(ent["fetch_kib"]))
        wk = float(np.median(ent["write_kib"]))
        ent["fetch_kib"] = fk
        ent["write_kib"] = wk
        ent["hbm_bytes_per_launch"] = fk * 1024.0 * out["fetch_factor"] + wk * 1024.0 * out["write_factor"]
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def counters_summarize(dbs, command: str):
    """Markdown table of the SQ / GRBM counters of the OMP kernels from
    rocprofv3 --pmc runs over --traffic-probe: per-wavefront instruction
    counts, and the matrix-core and VALU busy fractions over the launch:
    busy cycles summed over wavefronts / (SIMDs x launch cycles), the launch
    cycles being GRBM_GUI_ACTIVE / 8 (the counter adds up the 8 XCDs)."""
    import collections
    import sqlite3

    simds = 256 * 4
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for db in dbs:
        c = sqlite3.connect(db)
        for kn, cn, v in c.execute("select kernel_name, counter_name, sum(value) from counters_collection "
                                   "group by dispatch_id, counter_name"):
            if "k_omp_" in kn:
                per[kn.split("(")[0]][cn].append(float(v))
    lines = ["Command (on the MI355X machine; `$R` is the repository root), one run per counter set:", "", "```",
             command, "```", "",
             "Per launch (median over launches); per-wavefront figures divide by `SQ_WAVES`.  `SQ_*_CYCLES` and "
             "`SQ_ACTIVE_INST_*` count in units of 4 cycles except `SQ_VALU_MFMA_BUSY_CYCLES` (cycles).", ""]
    for kn, m in per.items():
        med = {cn: float(np.median(v)) for cn, v in m.items()}
        waves = med.get("SQ_WAVES", 1.0)
        lines.append(f"**`{kn}`** ({waves:.0f} wavefronts)")
        lines.append("")
        lines.append("| counter | per launch | per wavefront |")
        lines.append("|---|---:|---:|")
        for cn in sorted(med):
            lines.append(f"| `{cn}` | {med[cn]:.0f} | {med[cn] / waves:.1f} |")
        gui = med.get("GRBM_GUI_ACTIVE", 0.0) / 8
        if gui:
            lines.append(f"| launch cycles (GRBM_GUI_ACTIVE / 8) | {gui:.0f} | |")
            if "SQ_VALU_MFMA_BUSY_CYCLES" in med:
                lines.append(f"| matrix cores busy | {med['SQ_VALU_MFMA_BUSY_CYCLES'] / (simds * gui):.3f} | |")
            if "SQ_ACTIVE_INST_VALU" in med:
                lines.append(f"| VALU issuing | {4 * med['SQ_ACTIVE_INST_VALU'] / (simds * gui):.3f} | |")
        lines.append("")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-timeacc", action="store_true", help="skip the time versus accuracy studies")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-pipeline", action="store_true")
    ap.add_argument("--no-learning", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other configurations (FP64 denoising, 3-scale, video)")
    ap.add_argument("--serve-jobs", type=int, default=2000, help="Poisson arrivals per offered load")
    ap.add_argument("--serve-slots", type=int, default=4, help="server launches in flight")
    ap.add_argument("--serve-ring", type=int, default=8, help="client output sets (jobs outstanding)")
    ap.add_argument("--cpu-sample", type=int, default=65536,
                    help="patches of the workload the oracle is timed on")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="known-size elementwise pass plus cross-scale steps, for rocprofv3 --pmc")
    ap.add_argument("--traffic-summarize", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write profiles/traffic_<workload>.json from the two counter runs")
    ap.add_argument("--counters-summarize", nargs="+", metavar="DB",
                    help="markdown summary of SQ / GRBM counter runs over --traffic-probe")
    ap.add_argument("--traffic-command", default="",
                    help="the commands that produced the counter runs (recorded in the summary)")
    args = ap.parse_args()
    if args.traffic_probe:
        traffic_probe(args.workload)
        return
    if args.counters_summarize:
        counters_summarize(args.counters_summarize, args.traffic_command)
        return
    if args.traffic_summarize:
        traffic_summarize(args.traffic_summarize[0], args.traffic_summarize[1], args.workload,
                          args.traffic_command)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(every patch is independent: the batch would be split across GPUs, see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1511_05174_amd import cspd

    w = synth.make(args.workload)
    B = w.batch
    ks = list(w.k_scales)
    plan = cspd.plan_from_workload(w)
    tdt = torch.float64 if w.dtype == "f64" else torch.float32
    ndt = np.float64 if w.dtype == "f64" else np.float32
    dev = torch.device("cuda", 0)
    y = torch.from_numpy(np.ascontiguousarray(w.y.astype(ndt))).to(dev)
    mask = None if w.mask is None else torch.from_numpy(w.mask).to(dev)
    kf = None if w.k_fine is None else torch.from_numpy(w.k_fine.astype(np.int32)).to(dev)
    sup = torch.empty((B, plan.k_max), dtype=torch.int32, device=dev)
    coef = torch.empty((B, plan.k_max), dtype=tdt, device=dev)
    ku = torch.empty((B,), dtype=torch.int32, device=dev)
    xh = torch.empty((B, w.n), dtype=tdt, device=dev)
    stream = torch.cuda.current_stream()

    def cross_step():
        cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1], support=sup, coef=coef,
                                  k_used=ku, xhat=xh, stream=stream)

    def full_step():
        cspd.cspd_omp_full(plan, y, mask, kf, ks[-1], support=sup, coef=coef, k_used=ku, xhat=xh,
                           stream=stream)

    def timed(step, steps, warmup):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        cspd.cspd_profile_reset()
        cspd.cspd_profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cspd.cspd_profile_enable(False)
        prof = cspd.cspd_profile_read()
        return (t1 - t0) / steps, prof

    print(f"[bench] workload {args.workload}: B={B} dims={w.dims} atoms={w.atoms} K={ks} "
          f"phi={w.phi_kind} dtype={w.dtype}", file=sys.stderr, flush=True)
    t_cross, prof = timed(cross_step, args.steps, args.warmup)
    x_cross = xh.double().cpu().numpy()
    print(f"[bench] cross-scale: {t_cross * 1e3:.3f} ms/step", file=sys.stderr, flush=True)

    flops = kernel_flops(w, ks)
    # dominant kernel = largest summed duration over the timed region
    label, (launches, tot_ms) = max(prof.items(), key=lambda kv: kv[1][1])
    role = label.split(":")[-1]
    avg_ms = tot_ms / max(launches, 1)
    per_patch = flops.get(role)
    achieved = per_patch * B / (avg_ms * 1e-3) / 1e12 if per_patch else None
    traffic = load_traffic(args.workload, role, 1)
    peak = PEAK_FP32_VECTOR_TFLOPS if w.dtype == "f32" else PEAK_FP64_VECTOR_TFLOPS
    roofline = {
        "bound": bound_of(label),
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": None if achieved is None else achieved / peak,
        "traffic": traffic,
        "peak_unpacked_fp32": PEAK_FP32_VECTOR_UNPACKED_TFLOPS if w.dtype == "f32" else None,
        "frac_vs_unpacked_fp32": (None if achieved is None or w.dtype != "f32"
                                  else achieved / PEAK_FP32_VECTOR_UNPACKED_TFLOPS),
        "kernel": label,
        "kernel_ms": avg_ms,
        "flops_per_patch": per_patch,
        "kernels": {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)} for k, v in prof.items()},
    }

    full = None
    x_full = None
    if not args.no_full:
        try:
            t_full, prof_full = timed(full_step, max(1, args.steps // 4), 1)
            x_full = xh.double().cpu().numpy()
            full = {"value": B / t_full, "ms_per_step": t_full * 1e3,
                    "kernels": {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)}
                                for k, v in prof_full.items()}}
            print(f"[bench] full OMP: {t_full * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        except cspd.CspdError as e:
            print(f"[bench] full OMP unavailable: {e}", file=sys.stderr, flush=True)

    quality = {"psnr_db_cross": psnr_db(w.x, x_cross), "snr_db_cross": snr_db(w.x, x_cross)}
    if x_full is not None:
        quality["psnr_db_full"] = psnr_db(w.x, x_full)
        quality["snr_db_full"] = snr_db(w.x, x_full)

    # ---- equal PSNR (time-accuracy method of the paper's video experiment):
    # full OMP at several K, cross-scale at several (K_low, K_fine); for every
    # full operating point the cheapest cross-scale point within 0.1 dB.
    equal = None
    equal_d1 = None
    if full is not None and not args.no_sweep and w.n_scales == 2:
        equal = equal_psnr_phase(cspd, w, plan, timed)
        if args.workload == "c2":
            # the same sweep on the unmodified model dictionaries (child detail 1)
            import synth as _s
            w1 = _s.make("c2", detail=1.0)
            equal_d1 = equal_psnr_phase(cspd, w1, cspd.plan_from_workload(w1), timed)

    # ---- serving: Poisson arrivals of jobs of three shapes
    serving = None
    if not args.no_serve:
        serving = serve_phase(cspd, jobs=args.serve_jobs, slots=args.serve_slots, ring=args.serve_ring)
        print(f"[bench] serving capacity {serving['capacity_patches_per_s']:.3e} patches/s",
              file=sys.stderr, flush=True)

    # ---- batching: captured HIP graphs against eager calls
    graphs = None
    if not args.no_graph:
        graphs = graph_phase(cspd, w, ks)
        print(f"[bench] graphs: {json.dumps(graphs)}", file=sys.stderr, flush=True)

    # ---- batching: autotuned kernel per scale against the shape rules
    autotune = None
    if not args.no_autotune:
        autotune = autotune_phase(cspd, w, ks, y, mask, kf)
        print(f"[bench] autotune: {json.dumps(autotune)}", file=sys.stderr, flush=True)

    # ---- whole-image pipeline: patches -> zero-tree OMP -> averaging
    pipeline = None
    if not args.no_pipeline and args.workload == "c2":
        pipeline = pipeline_phase(cspd, w, ks)
        print(f"[bench] pipeline: {json.dumps(pipeline)}", file=sys.stderr, flush=True)

    # ---- dictionary learning (Section III-E): cross-scale vs plain K-SVD
    learning = None
    if not args.no_learning and args.workload == "c2":
        learning = learning_phase(cspd, w)
        print(f"[bench] learning: {json.dumps(learning)}", file=sys.stderr, flush=True)

    # ---- time versus accuracy: single-scale dictionaries of 256..8192 atoms
    # against zero-tree OMP on 8x8x32 video patches; the effect of Q
    time_accuracy = q_study = None
    if not args.no_timeacc:
        from paper_1511_05174_amd import timeacc
        time_accuracy = timeacc.video_time_accuracy(batch=1024, steps=2)
        z = time_accuracy["zero_tree"]
        print(f"[bench] time-accuracy: zero-tree {z['ms_per_call']:.3f} ms, {z['psnr_db']:.2f} dB; single-scale "
              + ", ".join(f"T{p['atoms']}/K{p['k']}: {p['ms_per_call']:.3f} ms {p['psnr_db']:.2f} dB"
                          for p in time_accuracy["single_scale"]), file=sys.stderr, flush=True)
        q_study = timeacc.q_effect()
        print(f"[bench] Q study: {json.dumps(q_study['points'])}", file=sys.stderr, flush=True)

    # ---- precision: bf16 / fp16 proxies with FP32 re-scoring (full OMP, 3-scale workload)
    precision = None
    if not args.no_precision:
        precision = precision_phase(cspd)
        print(f"[bench] precision: {json.dumps(precision)}", file=sys.stderr, flush=True)

    workloads = None
    if not args.no_workloads and args.workload == "c2":
        workloads = workloads_phase(cspd)

    cpu = None
    cpu1 = None
    if not args.no_cpu_baseline:
        import synth as _s
        import oracle
        oracle.build()
        n = min(args.cpu_sample, B)
        sub = _s.subset(w, np.arange(n))
        threads = len(os.sched_getaffinity(0))
        # the sample is solved repeatedly until about 10 s of wall time have
        # passed (a stable rate; each pass is the same work)
        reps = 0
        t0 = time.perf_counter()
        while True:
            oracle.omp_cross_scale(sub, n_threads=threads)
            reps += 1
            if time.perf_counter() - t0 >= 10.0 or reps >= 200:
                break
        t1 = time.perf_counter()
        cpu = {"value": n * reps / (t1 - t0), "unit": "patches/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n} patches of the workload, zero-tree OMP, FP64, solved {reps} times "
                         f"in {t1 - t0:.2f} s wall"}
        print(f"[bench] oracle: {n} patches x {reps} in {t1 - t0:.2f} s on {threads} threads",
              file=sys.stderr, flush=True)
        # the same oracle on one thread, over a smaller prefix (about 5 s)
        n1 = min(4096, n)
        sub1 = _s.subset(w, np.arange(n1))
        reps1 = 0
        t0 = time.perf_counter()
        while True:
            oracle.omp_cross_scale(sub1, n_threads=1)
            reps1 += 1
            if time.perf_counter() - t0 >= 5.0 or reps1 >= 200:
                break
        t1 = time.perf_counter()
        cpu1 = {"value": n1 * reps1 / (t1 - t0), "unit": "patches/s", "cores": 1, "kind": "oracle",
                "sample": f"first {n1} patches of the workload, zero-tree OMP, FP64, solved {reps1} times "
                          f"in {t1 - t0:.2f} s wall on one thread"}

    line = {
        "metric": "patches/sec cross-scale vs full OMP at equal PSNR; p50/p99 job latency",
        "value": B / t_cross,
        "unit": "patches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_cross * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.dtype == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {B} patches, dims {w.dims}, atoms {w.atoms}, "
                               f"K {ks}, phi {w.phi_kind}, {w.dtype}",
                   "patches": B, "parallelism": "none (1 GPU)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_1thread": cpu1,
        "workloads": workloads,
        "full_omp": full,
        "quality": quality,
        "equal_psnr": equal,
        "equal_psnr_child_detail_1": equal_d1,
        "serving": serving,
        "precision": precision,
        "time_accuracy": time_accuracy,
        "q_effect": q_study,
        "graphs": graphs,
        "autotune": autotune,
        "pipeline": pipeline,
        "learning": learning,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
