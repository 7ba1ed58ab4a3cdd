"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws random numbers and lays them out: dictionaries, the
measurement operator, sparse codes, clean signals, noise and masks.  It holds
none of the method's arithmetic (no correlation, selection or least squares);
both the FP64 oracle and the HIP path consume the arrays it returns.

Shapes follow the experiments of Section IV of the paper (8x8 image patches,
8x8x8 video patches, 5x5x4x4 light-field patches; fine dictionaries of up to
4096 atoms, coarse ones of 64-256) and the cross-scale model of Section III-A:
fine atom j is a child of coarse atom floor(j / Q) (the 0-based form of the
block map of Section III-B).  The paper's data sets and trained dictionaries
are not available; these inputs stand in for them.

Layout conventions (shared by every consumer):
  * ``dicts[s]`` has shape (T_s, N_s), C-contiguous: atom-contiguous, which is
    the column-major N_s x T_s dictionary D_s.
  * ``up_maps[s]`` (s < S-1) has length N_{s+1}; entry j is the scale-s
    coordinate that fine coordinate j of scale s+1 copies under the
    nearest-neighbour upsampler U (and averages into under the box
    downsampler W).
  * ``phi`` is row-major (M, N); ``y`` is (B, M); ``mask`` is (B, N) uint8.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# One seed per workload, as the workloads' recipe states.
SEEDS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5a": 51, "c5b": 52, "c5c": 53,
         "c4loc": 41, "bayer": 61, "lfca": 62}


@dataclass
class Workload:
    name: str
    seed: int
    dims: List[int]                 # N_s, coarse -> fine
    atoms: List[int]                # T_s
    dicts: List[np.ndarray]         # (T_s, N_s) float64
    up_maps: List[np.ndarray]       # length S-1, int32 arrays of length N_{s+1}
    phi_kind: str                   # "identity" | "dense" | "mask"
    m: int                          # measurement dimension
    phi: Optional[np.ndarray]       # (M, N) float64 or None
    x: np.ndarray                   # (B, N) clean signals
    y: np.ndarray                   # (B, M) measurements
    mask: Optional[np.ndarray]      # (B, N) uint8 or None
    k_scales: List[int]             # K per scale (finest entry = uniform K or max)
    k_fine: Optional[np.ndarray]    # (B,) int32 per-patch fine sparsity, or None
    sigma: float
    true_support: np.ndarray        # (B, Kmax) int32, fine indices, -1 padded
    dtype: str                      # "f64" | "f32"
    meta: dict = field(default_factory=dict)
    phase: Optional[np.ndarray] = None   # (B,) int32: each patch's operator when phi is (P, M, N)

    @property
    def n_scales(self) -> int:
        return len(self.dims)

    @property
    def n(self) -> int:
        return self.dims[-1]

    @property
    def batch(self) -> int:
        return self.y.shape[0]

    @property
    def q(self) -> List[int]:
        return [self.atoms[s] // self.atoms[s - 1] for s in range(1, self.n_scales)]


def _streams(seed: int, n: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(n)]


def box_map(fine_shape, factors) -> np.ndarray:
    """Up-map for a separable box down-sampler on a row-major grid.

    ``factors`` may hold an int (uniform block size along that axis) or an
    explicit list assigning each fine index along the axis to a coarse index.
    """
    axes = []
    coarse_shape = []
    for extent, f in zip(fine_shape, factors):
        if isinstance(f, (list, tuple, np.ndarray)):
            a = np.asarray(f, dtype=np.int64)
            assert a.shape == (extent,)
        else:
            assert extent % f == 0
            a = np.arange(extent) // f
        axes.append(a)
        coarse_shape.append(int(a.max()) + 1)
    grids = np.meshgrid(*axes, indexing="ij")
    idx = np.zeros(fine_shape, dtype=np.int64)
    for g, cs in zip(grids, coarse_shape):
        idx = idx * cs + g
    return idx.reshape(-1).astype(np.int32), tuple(coarse_shape)


def unit_columns(d: np.ndarray) -> np.ndarray:
    """Scale every atom (row of a (T, N) array) to unit Euclidean length."""
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def gaussian_dict(rng, t: int, n: int) -> np.ndarray:
    return unit_columns(rng.standard_normal((t, n)))


# Scale of the fine detail that children add to their upsampled parent.  At
# 0.5 the detail carries about a sixth of a child's energy (cosine between a
# child and its upsampled parent about 0.92): children resemble their parents,
# as the learned fine atoms of Section III do.  (At 1.0 the detail is as
# strong as the parent part and the coarse search under a pixel mask loses
# its parents much more often.)
CHILD_DETAIL = 0.5


def child_dict(rng, parent: np.ndarray, up_map: np.ndarray, q: int,
               detail: float = CHILD_DETAIL) -> np.ndarray:
    """Children that look like their upsampled parent plus detail that the box
    down-sampler removes, so W d_child is exactly proportional to d_parent.

    parent: (T_c, N_c); returns (T_c * q, N_f) with unit columns.
    """
    t_c, n_c = parent.shape
    n_f = up_map.shape[0]
    counts = np.bincount(up_map, minlength=n_c).astype(np.float64)
    up = parent[:, up_map] / np.sqrt(counts[up_map].mean())       # (T_c, N_f)
    g = rng.standard_normal((t_c * q, n_f))
    # remove the block mean of g: (I - U W) g
    block_sum = np.zeros((t_c * q, n_c))
    np.add.at(block_sum.T, up_map, g.T)
    g -= (block_sum / counts)[:, up_map]
    d = np.repeat(up, q, axis=0) + detail * g / np.sqrt(n_f)
    return unit_columns(d)


def _compose_maps(up_maps, dims):
    """maps[s][j] = scale-s coordinate of finest coordinate j."""
    s_count = len(dims)
    maps = [None] * s_count
    maps[-1] = np.arange(dims[-1], dtype=np.int64)
    for s in range(s_count - 2, -1, -1):
        maps[s] = up_maps[s].astype(np.int64)[maps[s + 1]]
    return maps


def draw_tree_support(rng, b: int, atoms, q, k_scales, k_fine=None):
    """Fine supports that obey the zero-tree rule: coarse support uniform,
    every finer support drawn without replacement from the children of the
    one above it.  Returns the finest support (B, Kmax), -1 padded."""
    s_count = len(atoms)
    kmax = int(k_fine.max()) if k_fine is not None else k_scales[-1]
    out = np.full((b, kmax), -1, dtype=np.int32)
    # scale 0
    keys = rng.random((b, atoms[0]))
    prev = np.argsort(keys, axis=1)[:, : k_scales[0]]
    for s in range(1, s_count):
        qs = q[s - 1]
        kids = (prev[:, :, None] * qs + np.arange(qs)[None, None, :]).reshape(b, -1)
        keys = rng.random(kids.shape)
        order = np.argsort(keys, axis=1)
        k_here = kmax if s == s_count - 1 else k_scales[s]
        k_here = min(k_here, kids.shape[1])
        prev = np.take_along_axis(kids, order[:, :k_here], axis=1)
    if s_count == 1:
        prev = prev
    if k_fine is not None:
        cols = np.arange(prev.shape[1])[None, :]
        prev = np.where(cols < k_fine[:, None], prev, -1)
    out[:, : prev.shape[1]] = prev
    return out


def synthesize(rng_coef, rng_noise, dict_f, support, phi_kind, phi, mask, sigma):
    b, kmax = support.shape
    n = dict_f.shape[1]
    coef = rng_coef.standard_normal((b, kmax))
    coef = np.where(support >= 0, coef, 0.0)
    x = np.zeros((b, n))
    for k in range(kmax):
        idx = support[:, k]
        valid = idx >= 0
        x[valid] += dict_f[idx[valid]] * coef[valid, k][:, None]
    if phi_kind == "identity":
        y = x + sigma * rng_noise.standard_normal(x.shape)
    elif phi_kind == "mask":
        y = (x + sigma * rng_noise.standard_normal(x.shape)) * mask
    elif phi.ndim == 3:
        # one operator per phase; ``mask`` carries the patches' phases here
        y = np.einsum("bmn,bn->bm", phi[mask], x)
        y = y + sigma * rng_noise.standard_normal(y.shape)
    else:
        y = x @ phi.T
        y = y + sigma * rng_noise.standard_normal(y.shape)
    return x, y


# ---- structured measurement operators (Section IV's acquisition models) ----

def bayer_mask(h: int, w: int) -> np.ndarray:
    """RGGB colour-filter array over an (h, w, 3) image: red at (even, even),
    green at (even, odd) and (odd, even), blue at (odd, odd); 1 = observed."""
    m = np.zeros((h, w, 3), dtype=np.uint8)
    m[0::2, 0::2, 0] = 1
    m[0::2, 1::2, 1] = 1
    m[1::2, 0::2, 1] = 1
    m[1::2, 1::2, 2] = 1
    return m


def coded_exposure_phases(rng, frames: int, patch: int, period: int) -> np.ndarray:
    """Location-dependent coded exposure: a per-pixel shutter code of
    ``period`` x ``period`` pixels (Bernoulli(1/2) per pixel and frame), tiled
    over the sensor.  A patch of patch x patch pixels starting at (y0, x0)
    sees the tile shifted by (y0 mod period, x0 mod period); each of the
    period^2 shifts is one operator, M = patch^2 rows over the frame-major
    (t, y, x) patch of N = frames * patch^2 samples: the coded image sums the
    open frames of each pixel.  Returns (period^2, patch^2, frames * patch^2)."""
    code = rng.integers(0, 2, size=(frames, period, period)).astype(np.float64)
    px = patch * patch
    ops = np.zeros((period * period, px, frames * px))
    yy, xx = np.meshgrid(np.arange(patch), np.arange(patch), indexing="ij")
    pix = (yy * patch + xx).reshape(-1)
    for dy in range(period):
        for dx in range(period):
            ph = dy * period + dx
            c = code[:, (yy + dy) % period, (xx + dx) % period].reshape(frames, px)
            for t in range(frames):
                ops[ph, pix, t * px + pix] = c[t]
    return ops


def coded_aperture_phi(rng, shots: int, ang=(4, 4), spatial=(8, 8)) -> np.ndarray:
    """Programmable-aperture light-field capture: each shot opens a binary
    code over the angular samples (Bernoulli(1/2)) and every pixel records
    the sum of its open views.  Rows (shot, y, x), columns (u, v, y, x)."""
    na, ns = ang[0] * ang[1], spatial[0] * spatial[1]
    codes = rng.integers(0, 2, size=(shots, na)).astype(np.float64)
    phi = np.zeros((shots * ns, na * ns))
    for s_ in range(shots):
        for a in range(na):
            phi[s_ * ns + np.arange(ns), a * ns + np.arange(ns)] = codes[s_, a]
    return phi


def make(name: str, batch: Optional[int] = None, seed: Optional[int] = None,
         dict_kind: str = "model", detail: float = CHILD_DETAIL) -> Workload:
    """Build one of the named workloads.

    c1: 2-scale FP64 denoising, 1024 patches, 8x8 -> 4x4, Dc 16x64, Df 64x256, Q 4.
    c2: 2-scale FP32 inpainting, 65536 patches, per-patch 50 % pixel mask,
        Dc 16x128, Df 64x1024, Q 8, K (4, 8).
    c3: 3-scale, 262144 patches, 16x16 -> 8x8 -> 4x4, dictionaries 16x64,
        64x512, 256x4096, Q 8, K (4, 8, 12), Gaussian Phi 128x256.
    c4: video 8x8x8 -> 4x4x2, 131072 patches, Dc 32x256, Df 512x4096, Q 16,
        coded-exposure Phi 64x512, per-patch K ~ U{4..16}, K_low 4.
    c5a/b/c: serving shapes (64-d / 512-d video / 400-d light field) with
        Gaussian Phi at 25 % measurement rate, K_fine ~ U{6..16}, K_low 4.

    ``detail`` scales the block-mean-free detail that model-consistent
    children add to their upsampled parent (CHILD_DETAIL by default).
    """
    name = name.lower()
    seed = SEEDS[name] if seed is None else seed
    r_dict, r_sup, r_coef, r_phi, r_noise, r_k, r_mask, r_extra = _streams(seed, 8)

    k_fine = None
    if name == "c1":
        b = 1024 if batch is None else batch
        up0, _ = box_map((8, 8), (2, 2))
        dims, atoms, ks, sigma, phi_kind, m, dtype = [16, 64], [64, 256], [4, 4], 0.01, "identity", 64, "f64"
        up_maps = [up0]
    elif name == "c2":
        b = 65536 if batch is None else batch
        up0, _ = box_map((8, 8), (2, 2))
        dims, atoms, ks, sigma, phi_kind, m, dtype = [16, 64], [128, 1024], [4, 8], 0.005, "mask", 64, "f32"
        up_maps = [up0]
    elif name == "c3":
        b = 262144 if batch is None else batch
        up0, _ = box_map((8, 8), (2, 2))
        up1, _ = box_map((16, 16), (2, 2))
        dims, atoms, ks, sigma, phi_kind, m, dtype = [16, 64, 256], [64, 512, 4096], [4, 8, 12], 0.005, "dense", 128, "f32"
        up_maps = [up0, up1]
    elif name == "c4":
        b = 131072 if batch is None else batch
        # frame-major (t, y, x) = (8, 8, 8) -> (2, 4, 4): blocks of 4 frames x 2 x 2 pixels
        up0, _ = box_map((8, 8, 8), (4, 2, 2))
        dims, atoms, ks, sigma, phi_kind, m, dtype = [32, 512], [256, 4096], [4, 16], 0.005, "dense", 64, "f32"
        up_maps = [up0]
        k_fine = r_k.integers(4, 17, size=b).astype(np.int32)
    elif name == "c4loc":
        # video coded exposure whose shutter tile differs with the patch position
        b = 32768 if batch is None else batch
        up0, _ = box_map((8, 8, 8), (4, 2, 2))
        dims, atoms, ks, sigma, phi_kind, m, dtype = [32, 512], [256, 4096], [4, 16], 0.005, "dense", 64, "f32"
        up_maps = [up0]
        k_fine = r_k.integers(4, 17, size=b).astype(np.int32)
    elif name == "bayer":
        # demosaicing: 24x24 RGB patches (y, x, c) over 12x12 per channel,
        # observed through the colour-filter array at the patch's position
        b = 4096 if batch is None else batch
        up0, _ = box_map((24, 24, 3), (2, 2, 1))
        dims, atoms, ks, sigma, phi_kind, m, dtype = [432, 1728], [128, 2048], [4, 8], 0.005, "mask", 1728, "f32"
        up_maps = [up0]
    elif name == "lfca":
        # light field 4x4 views x 8x8 pixels through two coded-aperture shots
        b = 16384 if batch is None else batch
        up0, _ = box_map((4, 4, 8, 8), (2, 2, 2, 2))
        dims, atoms, ks, sigma, phi_kind, m, dtype = [64, 1024], [128, 1024], [4, 8], 0.005, "dense", 128, "f32"
        up_maps = [up0]
    elif name in ("c5a", "c5b", "c5c"):
        b = 4096 if batch is None else batch
        if name == "c5a":
            up0, _ = box_map((8, 8), (2, 2))
            dims, atoms, m = [16, 64], [128, 1024], 16
        elif name == "c5b":
            up0, _ = box_map((8, 8, 8), (4, 2, 2))
            dims, atoms, m = [32, 512], [256, 4096], 128
        else:
            # angular 5 -> 2 with blocks {0,1,2}, {3,4}; spatial 4 -> 2
            ang = [0, 0, 0, 1, 1]
            up0, _ = box_map((5, 5, 4, 4), (ang, ang, 2, 2))
            dims, atoms, m = [16, 400], [256, 4096], 100
        ks, sigma, phi_kind, dtype = [4, 16], 0.005, "dense", "f32"
        up_maps = [up0]
        k_fine = r_k.integers(6, 17, size=b).astype(np.int32)
    else:
        raise ValueError(f"unknown workload {name!r}")

    s_count = len(dims)
    q = [atoms[s] // atoms[s - 1] for s in range(1, s_count)]
    # dictionaries
    dicts = [gaussian_dict(r_dict, atoms[0], dims[0])]
    for s in range(1, s_count):
        if dict_kind == "model":
            dicts.append(child_dict(r_dict, dicts[s - 1], up_maps[s - 1], q[s - 1], detail=detail))
        elif dict_kind == "indep":
            dicts.append(gaussian_dict(r_dict, atoms[s], dims[s]))
        else:
            raise ValueError(dict_kind)

    n = dims[-1]
    phi = None
    mask = None
    phase = None
    if name == "c4loc":
        phi = coded_exposure_phases(r_phi, 8, 8, 4)
        phase = r_extra.integers(0, phi.shape[0], size=b).astype(np.int32)
    elif name == "lfca":
        phi = coded_aperture_phi(r_phi, 2)
    elif name == "bayer":
        # patches cut at random positions: the CFA phase is the position's parity
        cfa = bayer_mask(2 * 24 + 2, 2 * 24 + 2)
        pos = r_mask.integers(0, 2, size=(b, 2))
        mask = np.stack([cfa[py:py + 24, px:px + 24].reshape(-1) for py, px in pos]).astype(np.uint8)
    elif phi_kind == "dense":
        if name == "c4":
            frames = r_phi.integers(0, 2, size=(8, 64)).astype(np.float64)
            phi = np.zeros((64, 512))
            for t in range(8):
                phi[np.arange(64), t * 64 + np.arange(64)] = frames[t]
        else:
            phi = r_phi.standard_normal((m, n)) / np.sqrt(m)
    elif phi_kind == "mask":
        mask = r_mask.integers(0, 2, size=(b, n)).astype(np.uint8)

    support = draw_tree_support(r_sup, b, atoms, q, ks, k_fine)
    x, y = synthesize(r_coef, r_noise, dicts[-1], support, phi_kind, phi,
                      phase if phase is not None else mask, sigma)
    return Workload(name=name, seed=seed, dims=dims, atoms=atoms, dicts=dicts, up_maps=up_maps,
                    phi_kind=phi_kind, m=m, phi=phi, x=x, y=y, mask=mask, k_scales=ks,
                    k_fine=k_fine, sigma=sigma, true_support=support, dtype=dtype,
                    meta={"dict_kind": dict_kind, "child_detail": detail}, phase=phase)


def custom(dims, atoms, batch, seed, phi_kind="identity", m=None, k_scales=None, sigma=0.0,
           up_maps=None, dict_kind="indep", k_fine=None, dtype="f64") -> Workload:
    """A small workload with explicit shapes, used by edge-case and parity tests.

    When ``up_maps`` is None each scale's coordinates map to the coarser one by
    integer division (j -> j * N_s // N_{s+1}), which is a valid box map when
    the dimensions divide.
    """
    s_count = len(dims)
    r_dict, r_sup, r_coef, r_phi, r_noise, r_k, r_mask, _ = _streams(seed, 8)
    if up_maps is None:
        up_maps = [(np.arange(dims[s + 1]) * dims[s] // dims[s + 1]).astype(np.int32)
                   for s in range(s_count - 1)]
    q = [atoms[s] // atoms[s - 1] for s in range(1, s_count)]
    dicts = [gaussian_dict(r_dict, atoms[0], dims[0])]
    for s in range(1, s_count):
        if dict_kind == "model":
            dicts.append(child_dict(r_dict, dicts[s - 1], up_maps[s - 1], q[s - 1]))
        else:
            dicts.append(gaussian_dict(r_dict, atoms[s], dims[s]))
    n = dims[-1]
    if k_scales is None:
        k_scales = [min(2, atoms[0])] + [2] * (s_count - 1)
    phi = None
    mask = None
    if phi_kind == "dense":
        m = m or max(1, n // 2)
        phi = r_phi.standard_normal((m, n)) / np.sqrt(m)
    else:
        m = n
        if phi_kind == "mask":
            mask = r_mask.integers(0, 2, size=(batch, n)).astype(np.uint8)
    support = draw_tree_support(r_sup, batch, atoms, q, k_scales, k_fine)
    x, y = synthesize(r_coef, r_noise, dicts[-1], support, phi_kind, phi, mask, sigma)
    return Workload(name="custom", seed=seed, dims=list(dims), atoms=list(atoms), dicts=dicts,
                    up_maps=up_maps, phi_kind=phi_kind, m=m, phi=phi, x=x, y=y, mask=mask,
                    k_scales=list(k_scales), k_fine=k_fine, sigma=sigma, true_support=support,
                    dtype=dtype, meta={"dict_kind": dict_kind})


def subset(w: Workload, idx) -> Workload:
    """The same workload restricted to the patches ``idx`` (dictionaries shared)."""
    idx = np.asarray(idx)
    return Workload(name=w.name, seed=w.seed, dims=w.dims, atoms=w.atoms, dicts=w.dicts,
                    up_maps=w.up_maps, phi_kind=w.phi_kind, m=w.m, phi=w.phi, x=w.x[idx],
                    y=w.y[idx], mask=None if w.mask is None else w.mask[idx],
                    k_scales=w.k_scales, k_fine=None if w.k_fine is None else w.k_fine[idx],
                    sigma=w.sigma, true_support=w.true_support[idx], dtype=w.dtype,
                    meta=dict(w.meta, subset=True), phase=None if w.phase is None else w.phase[idx])
