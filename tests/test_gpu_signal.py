"""Whole-signal patch kernels on the GPU against the patch oracle
(oracle/signal.py), and an inpainting pipeline (patches -> zero-tree OMP ->
averaging) checked stage by stage (MI355X only).

Extraction is a copy: bit-exact.  Aggregation sums in FP64 in grid order as
the oracle does and rounds once to FP32: within one FP32 rounding."""
import numpy as np
import pytest

import gpu_util as G
import parity
import synth
from oracle import signal as S
from paper_1511_05174_amd import cspd

pytestmark = pytest.mark.gpu

CASES = [((37, 53), (8, 8), (3, 5)), ((64, 64), (8, 8), (8, 8)), ((12, 16, 17), (4, 8, 8), (4, 3, 2)),
         ((5, 5, 11, 13), (5, 5, 4, 4), (1, 1, 3, 2)), ((100,), (16,), (7,))]


@pytest.mark.parametrize("shape,patch,stride", CASES)
def test_extract_matches_oracle(shape, patch, stride):
    torch = G.torch_mod()
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape).astype(np.float32)
    m = (rng.random(shape) < 0.5).astype(np.uint8)
    grid = cspd.patch_grid(shape, patch, stride)
    y, pm = cspd.cspd_extract_patches(grid, torch.from_numpy(x).cuda(), torch.from_numpy(m).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), S.extract(x, patch, stride))
    assert np.array_equal(pm.cpu().numpy(), S.extract(m, patch, stride))
    y2, pm2 = cspd.cspd_extract_patches(grid, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(y2.cpu().numpy(), y.cpu().numpy()) and int(pm2.min()) == 1


@pytest.mark.parametrize("shape,patch,stride", CASES)
def test_aggregate_matches_oracle(shape, patch, stride):
    torch = G.torch_mod()
    grid = cspd.patch_grid(shape, patch, stride)
    n = cspd.cspd_patch_count(grid)
    est = np.random.default_rng(2).standard_normal((n, int(np.prod(patch)))).astype(np.float32)
    out = cspd.cspd_aggregate_patches(grid, torch.from_numpy(est).cuda())
    torch.cuda.synchronize()
    ref = S.aggregate(est, shape, patch, stride).astype(np.float32)
    assert np.array_equal(out.cpu().numpy(), ref)


def test_inpainting_pipeline_stages():
    """A 96 x 104 image with half of its pixels removed: patches of 8 x 8 at
    stride 4 through the inpainting plan's zero-tree OMP, then averaging.
    Each stage against the oracle on the GPU stage's own input."""
    torch = G.torch_mod()
    w = synth.make("c2", batch=16)                       # the inpainting dictionaries (8x8 / 4x4)
    plan = cspd.plan_from_workload(w)
    rng = np.random.default_rng(3)
    shape, patch, stride = (96, 104), (8, 8), (4, 4)
    # image: averaged overlapping dictionary patches (smooth at patch scale)
    grid = cspd.patch_grid(shape, patch, stride)
    n = cspd.cspd_patch_count(grid)
    src = synth.make("c2", batch=n, seed=31)
    clean = S.aggregate(src.x, shape, patch, stride).astype(np.float32)
    mask = (rng.random(shape) < 0.5).astype(np.uint8)
    meas = (clean * mask).astype(np.float32)
    y, pm = cspd.cspd_extract_patches(grid, torch.from_numpy(meas).cuda(), torch.from_numpy(mask).cuda())
    sup, coef, ku, xh = cspd.cspd_omp_cross_scale(plan, y, pm, w.k_scales[:-1], None, w.k_scales[-1])
    img = cspd.cspd_aggregate_patches(grid, xh)
    torch.cuda.synchronize()
    yh, pmh, xhh = y.cpu().numpy(), pm.cpu().numpy(), xh.cpu().numpy()
    assert np.array_equal(yh, S.extract(meas, patch, stride))
    assert np.array_equal(pmh, S.extract(mask, patch, stride))
    # OMP stage: the extracted patches as a workload, against the oracle
    import dataclasses
    wp = dataclasses.replace(w, y=yh.astype(np.float64), mask=pmh, x=np.zeros((n, w.n)), k_fine=None,
                             true_support=np.repeat(w.true_support[:1], n, axis=0))
    gs = parity.gpu_scales(wp, sup.cpu().numpy(), ku.cpu().numpy())
    rep = parity.compare(wp, gs, coef.double().cpu().numpy(), ku.cpu().numpy(), xh.double().cpu().numpy(),
                         tie_tol=1e-6)
    print(f"[pipeline omp] {rep.summary()}", flush=True)
    rep.check(1e-5, 1e-5)
    # averaging stage
    assert np.array_equal(img.cpu().numpy(), S.aggregate(xhh, shape, patch, stride).astype(np.float32))
    err = float(np.sqrt(np.mean((img.cpu().numpy() - clean) ** 2)) / np.sqrt(np.mean(clean ** 2)))
    print(f"[pipeline] relative error of the inpainted image {err:.3f}", flush=True)
    assert np.isfinite(err)


PAPER_SHAPES = [
    # name: signal shape, patch, stride, box factors, atoms (coarse, fine)
    ("rgb24_overlap18", (60, 66, 3), (24, 24, 3), (6, 6, 3), (2, 2, 1), (128, 2048)),
    ("video_8x8x32", (36, 20, 20), (32, 8, 8), (4, 4, 4), (2, 2, 2), (64, 1024)),
    ("lightfield_4x4x8x8", (4, 4, 20, 20), (4, 4, 8, 8), (1, 1, 4, 4), (2, 2, 2, 2), (64, 1024)),
]


@pytest.mark.parametrize("name,shape,patch,stride,box,atoms", PAPER_SHAPES)
def test_denoising_pipeline_at_the_paper_shapes(name, shape, patch, stride, box, atoms):
    """Denoising of a whole signal at the paper's patch shapes (Section IV: 24x24
    RGB image patches with an overlap of 18, 8x8x32 video patches, 4x4 views
    of 8x8 pixels): patches -> zero-tree OMP -> averaging, each stage against
    the oracle on the GPU stage's own input."""
    torch = G.torch_mod()
    up, coarse = synth.box_map(patch, box)
    dims = [int(np.prod(coarse)), int(np.prod(patch))]
    grid = cspd.patch_grid(shape, patch, stride)
    n = cspd.cspd_patch_count(grid)
    w = synth.custom(dims, list(atoms), n, seed=91, k_scales=[4, 8], sigma=0.0, up_maps=[up],
                     dict_kind="model", dtype="f32")
    plan = cspd.plan_from_workload(w)
    clean = S.aggregate(w.x, shape, patch, stride).astype(np.float32)
    rng = np.random.default_rng(4)
    sigma = 0.1 * float(np.sqrt(np.mean(clean ** 2)))
    noisy = (clean + sigma * rng.standard_normal(shape)).astype(np.float32)
    y, _ = cspd.cspd_extract_patches(grid, torch.from_numpy(noisy).cuda(), want_mask=False)
    sup, coef, ku, xh = cspd.cspd_omp_cross_scale(plan, y, None, w.k_scales[:-1], None, w.k_scales[-1])
    img = cspd.cspd_aggregate_patches(grid, xh)
    torch.cuda.synchronize()
    yh, xhh = y.cpu().numpy(), xh.cpu().numpy()
    assert np.array_equal(yh, S.extract(noisy, patch, stride))
    import dataclasses
    wp = dataclasses.replace(w, y=yh.astype(np.float64), x=np.zeros((n, w.n)), k_fine=None)
    gs = parity.gpu_scales(wp, sup.cpu().numpy(), ku.cpu().numpy())
    rep = parity.compare(wp, gs, coef.double().cpu().numpy(), ku.cpu().numpy(), xh.double().cpu().numpy(),
                         tie_tol=1e-6)
    print(f"[{name} omp, {n} patches of {w.n}] {rep.summary()}", flush=True)
    rep.check(1e-5, 1e-5)
    assert np.array_equal(img.cpu().numpy(), S.aggregate(xhh, shape, patch, stride).astype(np.float32))
    e_noisy = float(np.sqrt(np.mean((noisy - clean) ** 2)))
    e_out = float(np.sqrt(np.mean((img.cpu().numpy() - clean) ** 2)))
    # (a signal averaged from overlapping model patches is not sparse in every
    # window, so no quality bar is set here; the stages are what is checked)
    print(f"[{name}] rms error: noisy {e_noisy:.4f}, estimate {e_out:.4f}", flush=True)
    assert np.isfinite(e_out)
