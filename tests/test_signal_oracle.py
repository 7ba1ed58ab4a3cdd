"""Pins of the whole-signal patch oracle (oracle/signal.py): hand-worked
grids and averages, and invariants that hold for any signal (CPU only)."""
import numpy as np
import pytest

from oracle import signal as S
from paper_1511_05174_amd import cspd


def test_grid_positions_hand_worked():
    assert S.grid_positions(5, 3, 2) == [0, 2]           # regular grid reaches the end
    assert S.grid_positions(6, 3, 2) == [0, 2, 3]        # one more, aligned to the end
    assert S.grid_positions(8, 8, 3) == [0]              # a single patch
    assert S.grid_positions(10, 4, 4) == [0, 4, 6]
    with pytest.raises(ValueError):
        S.grid_positions(3, 4, 1)


def test_extract_hand_worked_1d_and_2d():
    x = np.arange(6.0)
    p = S.extract(x, [3], [2])
    assert p.tolist() == [[0, 1, 2], [2, 3, 4], [3, 4, 5]]
    img = np.arange(20.0).reshape(4, 5)                  # (y, x)
    q = S.extract(img, [2, 3], [2, 2])                   # y positions [0, 2]; x positions [0, 2]
    assert q.shape == (4, 6)
    # patch 1 = grid (0, 1): rows 0..1, columns 2..4, row-major inside the patch
    assert q[1].tolist() == [2, 3, 4, 7, 8, 9]
    # patch 2 = grid (1, 0): rows 2..3, columns 0..2
    assert q[2].tolist() == [10, 11, 12, 15, 16, 17]


def test_aggregate_hand_worked_1d():
    est = np.array([[1.0, 2.0, 3.0], [10.0, 20.0, 30.0], [100.0, 200.0, 300.0]])
    out = S.aggregate(est, [6], [3], [2])                # starts 0, 2, 3
    # sample 2: patches 0 (3.0) and 1 (10.0); sample 3: patches 1 (20.0) and 2 (100.0)
    # sample 4: patches 1 (30.0) and 2 (200.0); sample 5: patch 2 (300.0)
    assert np.allclose(out, [1.0, 2.0, 6.5, 60.0, 115.0, 300.0], rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape,patch,stride", [((13, 17), (4, 5), (3, 2)), ((6, 9, 7), (2, 4, 3), (1, 3, 2)),
                                                ((5, 5, 6, 7), (3, 2, 4, 4), (2, 2, 1, 3))])
def test_aggregate_of_extract_is_identity(shape, patch, stride):
    x = np.random.default_rng(0).standard_normal(shape)
    y = S.aggregate(S.extract(x, patch, stride), shape, patch, stride)
    assert np.allclose(y, x, rtol=1e-14, atol=1e-14)


def test_coverage_counts():
    ones = S.extract(np.ones((9, 9)), [3, 3], [3, 3])
    assert ones.shape == (9, 9)                           # non-overlapping: 9 patches of 9
    cnt = S.aggregate(np.arange(1, 10, dtype=float)[:, None] * np.ones((9, 9)), [9, 9], [3, 3], [3, 3])
    assert np.array_equal(cnt[0:3, 0:3], np.full((3, 3), 1.0))
    assert np.array_equal(cnt[6:9, 6:9], np.full((3, 3), 9.0))


def test_library_grid_count_matches_oracle():
    """The library's patch count (host-side grid arithmetic, no device)."""
    for shape, patch, stride in [((13, 17), (4, 5), (3, 2)), ((6, 9, 7), (2, 4, 3), (1, 3, 2)), ((64,), (8,), (8,))]:
        n = len(S.extract(np.zeros(shape), patch, stride))
        assert cspd.cspd_patch_count(cspd.patch_grid(shape, patch, stride)) == n
    with pytest.raises(cspd.CspdError):
        cspd.cspd_patch_count(cspd.patch_grid((4, 4), (5, 2), (1, 1)))
    with pytest.raises(cspd.CspdError):
        cspd.cspd_patch_count(cspd.patch_grid((4, 4), (2, 2), (0, 1)))
