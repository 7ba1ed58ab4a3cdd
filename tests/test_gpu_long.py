"""Long candidate vectors (more than 256 coordinates) against the FP64 oracle
(MI355X only): the patch shapes of the paper's experiments (Section IV) --
24x24 image patches over 12x12, 8x8x32 video patches over 4x4x16, 4x4x8x8
light-field patches over 2x2x4x4 -- under the identity, a per-patch pixel
mask and a shared dense operator, zero-tree OMP and full OMP.  Under a
per-patch mask the long-vector kernel runs; under a shared operator the
finest scale runs in coefficient coordinates on the plan's Gram table.  Dictionaries
are smaller than the paper's (hundreds of atoms, not 8192) so that the
oracle finishes in seconds; the kernel is the same for any atom count up to
its candidate cap.
"""
import numpy as np
import pytest

import gpu_util as G
import synth
from paper_1511_05174_amd import cspd
from test_gpu_parity import check_cross, check_full

pytestmark = pytest.mark.gpu

SHAPES = {
    # name: (fine grid, box factors)
    "img24": ((24, 24), (2, 2)),
    "vid32": ((32, 8, 8), (2, 2, 2)),     # frame-major (t, y, x)
    "lf": ((4, 4, 8, 8), (2, 2, 2, 2)),   # (u, v, y, x)
}


def long_workload(shape, batch, seed, atoms=(64, 512), ks=(3, 6), phi_kind="identity", m=None):
    grid, f = SHAPES[shape]
    up, coarse = synth.box_map(grid, f)
    dims = [int(np.prod(coarse)), int(np.prod(grid))]
    return synth.custom(dims, list(atoms), batch, seed, phi_kind=phi_kind, m=m, k_scales=list(ks),
                        sigma=0.01, up_maps=[up], dict_kind="model", dtype="f32")


def _kernels(plan, w):
    """Run once with event recording on; the kernel labels that ran."""
    cspd.cspd_profile_reset()
    cspd.cspd_profile_enable(True)
    G.run_cross(plan, w)
    cspd.cspd_profile_enable(False)
    return sorted(cspd.cspd_profile_read())


@pytest.mark.parametrize("shape,phi_kind,atoms,ks,batch", [
    ("img24", "identity", (64, 512), (3, 6), 301),
    ("img24", "mask", (64, 512), (3, 6), 257),
    ("vid32", "identity", (64, 1024), (4, 8), 129),
    ("lf", "mask", (64, 512), (4, 8), 200),
    # 70 candidates at the finest scale (above the Gram mode's 64): the
    # proxy loop, its candidate groups ragged at the end of the list
    ("img24", "mask", (64, 640), (7, 6), 173),
    # 128 first-scale candidates over 2x2 blocks of a random mask (blocks
    # with nothing observed weigh 0): the proxy loop's small instance
    ("img24", "mask", (128, 1024), (3, 6), 150),
])
def test_long_cross(shape, phi_kind, atoms, ks, batch):
    w = long_workload(shape, batch, seed=31, atoms=atoms, ks=ks, phi_kind=phi_kind)
    print(f"long cross: {shape} {phi_kind} dims {w.dims} atoms {w.atoms} K {ks} B {batch}", flush=True)
    check_cross(w)
    labels = _kernels(cspd.plan_from_workload(w), w)
    want = "omp_long<" if phi_kind == "mask" else "omp_batch<f32,c"
    assert any(l.startswith(want) and l.endswith(":s1") for l in labels), labels


def test_long_dense_operator_every_scale():
    """A shared Gaussian operator with 512 measurements of a 1024-sample
    light field: every scale's effective vectors have 512 coordinates (the
    first on the long-vector kernel, the finest on the Gram table)."""
    w = long_workload("lf", 160, seed=32, atoms=(32, 256), ks=(3, 6), phi_kind="dense", m=512)
    check_cross(w)
    labels = _kernels(cspd.plan_from_workload(w), w)
    assert any(l.startswith("omp_long<") and l.endswith(":s0") for l in labels), labels
    assert any(l.startswith("omp_batch<f32,c") and l.endswith(":s1") for l in labels), labels


def test_long_full_search():
    """Algorithm 1 over every atom of a 576-coordinate dictionary."""
    w = synth.custom([576], [384], 200, seed=33, k_scales=[6], sigma=0.01, dtype="f32")
    check_full(w)


def test_long_ragged_sparsity_and_capped_candidates():
    """Per-patch fine sparsity (some above the candidate count, some zero)."""
    w = long_workload("img24", 190, seed=34, atoms=(32, 256), ks=(2, 16))
    rng = np.random.default_rng(3)
    kf = rng.integers(0, 17, size=w.batch).astype(np.int32)
    import dataclasses
    w = dataclasses.replace(w, k_fine=kf)
    check_cross(w)


def test_long_vectors_several_operators():
    """Three dense operators of 512 measurements over 1,024-sample light-field
    patches, one per patch: every scale's effective vectors have 512
    coordinates, so the long-vector kernel runs each patch on its own
    operator's candidates (the Gram mode at the first scale's 32 atoms, the
    proxy loop above 64 candidates)."""
    import dataclasses
    from test_gpu_operators import run_phased
    import parity
    from test_gpu_parity import TOL
    w = long_workload("lf", 150, seed=35, atoms=(32, 512), ks=(5, 8), phi_kind="dense", m=512)
    rng = np.random.default_rng(8)
    phis = np.stack([w.phi * rng.choice([-1.0, 1.0], size=(1, w.phi.shape[1])) for _ in range(3)])
    ph = rng.integers(0, 3, size=w.batch).astype(np.int32)
    w2 = dataclasses.replace(w, phi=phis, phase=ph)
    plan = cspd.plan_from_workload(w2)
    out = run_phased(plan, w2)
    ks = w2.k_scales
    wo = G.with_y(w2, out["y64"])
    sup = parity.gpu_scales(w2, out["support"], out["k_used"], out["support_coarse"], ks[:-1])
    rep = parity.compare(wo, sup, out["coef"], out["k_used"], out["xhat"], k_scales=ks, tie_tol=TOL["f32"]["tie"])
    print(f"[3 operators, 512 measurements, B={w2.batch}] {rep.summary()}", flush=True)
    rep.check(TOL["f32"]["coef"], TOL["f32"]["xhat"])
    cspd.cspd_profile_reset()
    cspd.cspd_profile_enable(True)
    run_phased(plan, w2)
    cspd.cspd_profile_enable(False)
    labels = sorted(cspd.cspd_profile_read())
    assert any(l.startswith("omp_long<f32,gram,") and l.endswith(":s0") for l in labels), labels
    assert any(l.startswith("omp_long<f32,lp") and l.endswith(":s1") for l in labels), labels
