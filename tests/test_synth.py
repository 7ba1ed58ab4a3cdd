"""The seeded generator: shapes, reproducibility and the model properties the
cross-scale dictionaries must have (Section III-A)."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5a", "c5b", "c5c"])
def test_shapes_and_seed(name):
    w = synth.make(name, batch=64)
    again = synth.make(name, batch=64)
    assert np.array_equal(w.y, again.y) and np.array_equal(w.dicts[-1], again.dicts[-1])
    assert w.y.shape == (64, w.m)
    for s in range(w.n_scales):
        assert w.dicts[s].shape == (w.atoms[s], w.dims[s])
        np.testing.assert_allclose(np.linalg.norm(w.dicts[s], axis=1), 1.0, rtol=1e-12)
    for s in range(1, w.n_scales):
        assert w.atoms[s] % w.atoms[s - 1] == 0
        up = w.up_maps[s - 1]
        assert up.shape == (w.dims[s],) and up.min() == 0 and up.max() == w.dims[s - 1] - 1


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5c"])
def test_down_up_is_identity(name):
    """W (block mean) after U (replication) is the identity on the coarse space."""
    w = synth.make(name, batch=4)
    for s in range(1, w.n_scales):
        up = w.up_maps[s - 1]
        v = np.random.default_rng(0).standard_normal(w.dims[s - 1])
        uv = v[up]
        counts = np.bincount(up, minlength=w.dims[s - 1])
        wuv = np.bincount(up, weights=uv, minlength=w.dims[s - 1]) / counts
        np.testing.assert_allclose(wuv, v, rtol=1e-13)


@pytest.mark.parametrize("name", ["c1", "c3", "c4"])
def test_children_predict_parent(name):
    """Model dictionaries: the box average of a child is parallel to its parent
    (fine atom j is a child of coarse atom floor(j / Q))."""
    w = synth.make(name, batch=4)
    for s in range(1, w.n_scales):
        up = w.up_maps[s - 1]
        q = w.atoms[s] // w.atoms[s - 1]
        counts = np.bincount(up, minlength=w.dims[s - 1])
        for j in range(0, w.atoms[s], max(1, w.atoms[s] // 50)):
            child = w.dicts[s][j]
            wc = np.bincount(up, weights=child, minlength=w.dims[s - 1]) / counts
            parent = w.dicts[s - 1][j // q]
            cos = abs(wc @ parent) / np.linalg.norm(wc)
            assert cos > 1 - 1e-12


def test_true_support_is_a_tree():
    w = synth.make("c3", batch=256)
    q = w.atoms[2] // w.atoms[1]
    assert np.all(w.true_support[:, :12] >= 0)
    # all fine atoms descend from at most K_mid mid-scale atoms
    parents = w.true_support // q
    assert max(len(set(r)) for r in parents) <= 8


def test_uneven_sparsity():
    w = synth.make("c4", batch=1000)
    assert w.k_fine.min() >= 4 and w.k_fine.max() <= 16
    assert set(np.unique(w.k_fine)) == set(range(4, 17))
    nz = (w.true_support >= 0).sum(axis=1)
    assert np.array_equal(nz, w.k_fine)


def test_mask_noise_only_on_observed():
    w = synth.make("c2", batch=128)
    assert np.all(w.y[w.mask == 0] == 0)
    assert 0.4 < w.mask.mean() < 0.6


def test_coded_exposure_operator():
    w = synth.make("c4", batch=2)
    phi = w.phi
    assert phi.shape == (64, 512)
    # each measurement pixel p sums frames t where that frame's mask is on
    for p in range(64):
        cols = np.flatnonzero(phi[p])
        assert np.all(cols % 64 == p)
    assert set(np.unique(phi)) <= {0.0, 1.0}
