"""Pins of the K-SVD dictionary-update oracle (oracle/ksvd.py), from
properties the update must have rather than from its own formula (CPU)."""
import numpy as np

from oracle import ksvd


def _random_problem(rng, P=60, N=8, T=10, K=3):
    D = rng.standard_normal((T, N))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    sup = np.full((P, K + 1), -1, dtype=np.int32)
    coef = np.zeros((P, K + 1))
    for p in range(P):
        a = rng.choice(T - 1, size=K, replace=False)      # atom T-1 is never used
        sup[p, :K] = a
        coef[p, :K] = rng.standard_normal(K)
    X = rng.standard_normal((P, N))
    return X, D, sup, coef


def test_error_never_increases_and_atoms_stay_unit():
    rng = np.random.default_rng(0)
    X, D, sup, coef = _random_problem(rng)
    before = np.linalg.norm(ksvd.residual(X, D, sup, coef))
    D1, c1, R1 = ksvd.update(X, D, sup, coef)
    after = np.linalg.norm(R1)
    assert after <= before + 1e-12
    assert np.allclose(np.linalg.norm(D1, axis=1), 1.0)
    assert np.array_equal(D1[-1], D[-1])                  # unused atom unchanged
    assert np.allclose(R1, ksvd.residual(X, D1, sup, c1))  # the returned residual is the residual


def test_exact_rank_one_error_is_recovered():
    rng = np.random.default_rng(1)
    N, P = 6, 20
    a = rng.standard_normal(N)
    a /= np.linalg.norm(a)
    b = rng.standard_normal(P)
    X = np.outer(b, a)                                    # every signal is a multiple of a
    D = rng.standard_normal((2, N))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    sup = np.array([[0]] * P, dtype=np.int32)             # only atom 0 is used
    coef = rng.standard_normal((P, 1))
    D1, c1, R1 = ksvd.update(X, D, sup, coef)
    sgn = 1.0 if a @ D[0] >= 0 else -1.0
    assert np.allclose(D1[0], sgn * a)
    assert np.allclose(c1[:, 0], sgn * b)
    assert np.allclose(R1, 0.0, atol=1e-12)


def test_single_user_takes_its_error_vector():
    """One signal using atoms 0 and 2: atom 0 (updated first) becomes the
    normalised error without it, its coefficient that error's norm."""
    rng = np.random.default_rng(2)
    N = 5
    X = rng.standard_normal((1, N))
    D = rng.standard_normal((3, N))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    sup = np.array([[0, 2]], dtype=np.int32)
    coef = rng.standard_normal((1, 2))
    e = X[0] - coef[0, 1] * D[2]
    D1, c1, _ = ksvd.update(X, D, sup, coef)
    sgn = 1.0 if e @ D[0] >= 0 else -1.0
    assert np.allclose(D1[0], sgn * e / np.linalg.norm(e))
    assert np.isclose(c1[0, 0], sgn * np.linalg.norm(e))


def test_planted_dictionary_is_recovered_with_true_supports():
    rng = np.random.default_rng(3)
    N, T, K, P = 12, 16, 3, 800
    Dt = rng.standard_normal((T, N))
    Dt /= np.linalg.norm(Dt, axis=1, keepdims=True)
    sup = np.stack([rng.choice(T, size=K, replace=False) for _ in range(P)]).astype(np.int32)
    ct = rng.standard_normal((P, K))
    X = np.stack([ct[p] @ Dt[sup[p]] for p in range(P)])
    D = Dt + 0.2 * rng.standard_normal((T, N))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    coef = np.stack([np.linalg.lstsq(D[sup[p]].T, X[p], rcond=None)[0] for p in range(P)])
    for _ in range(30):
        D, coef, R = ksvd.update(X, D, sup, coef)
    cos = np.abs(np.sum(D * Dt, axis=1))
    assert cos.min() > 0.999, cos.min()
    assert np.linalg.norm(R) < 1e-2 * np.linalg.norm(X)


def test_init_children_draws_from_parent_users():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((50, 8))
    coarse = np.full((50, 2), -1, dtype=np.int32)
    coarse[:10, 0] = 1                                     # signals 0..9 use coarse atom 1
    D = ksvd.init_children(X, coarse, q=3, t_low=2, rng=np.random.default_rng(5))
    assert D.shape == (6, 8) and np.allclose(np.linalg.norm(D, axis=1), 1.0)
    Xn = X / np.linalg.norm(X, axis=1, keepdims=True)
    for c in range(3):                                     # children of atom 1 come from signals 0..9
        assert np.min(np.linalg.norm(Xn[:10] - D[3 + c], axis=1)) < 1e-12


def test_unused_atoms_take_the_least_represented_signals():
    """Heuristic 3 (Section III-G), worked by hand: atoms 1 and 3 have no user;
    errors [0.1, 0.5, 0.5, 0.2] -> atom 1 takes signal 1 (largest error, lower
    index of the tie), atom 3 takes signal 2 (signal 1 is taken)."""
    X = np.array([[3.0, 4.0], [0.0, 2.0], [1.0, 0.0], [1.0, 1.0]])
    D = np.array([[1.0, 0.0], [0.0, 1.0], [0.6, 0.8], [0.8, 0.6]])
    sup = np.array([[0, -1], [2, -1], [0, 2], [2, -1]], dtype=np.int32)
    err = np.array([0.1, 0.5, 0.5, 0.2])
    D2, rep = ksvd.replace_unused(D, X, sup, err)
    assert rep == [1, 3]
    assert np.allclose(D2[1], [0.0, 1.0]) and np.allclose(D2[3], [1.0, 0.0])
    assert np.array_equal(D2[[0, 2]], D[[0, 2]])


def test_unused_children_draw_from_their_parents_signals():
    """Heuristic 4: a fine atom is replaced from the signals whose coarse
    support holds its parent; with no such signal, from all."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((6, 4))
    coarse = np.array([[0], [1], [0], [1], [1], [0]])
    sup = np.array([[0], [2], [0], [3], [2], [0]], dtype=np.int32)   # atoms 1 (parent 0), 4, 5 (parent 2) unused
    err = np.array([0.3, 0.9, 0.1, 0.2, 0.8, 0.4])
    D = np.eye(6, 4)
    D2, rep = ksvd.replace_unused(D, X, sup, err, coarse_support=coarse, q=2)
    assert rep == [1, 4, 5]
    # atom 1 (parent 0): signals 0, 2, 5 -> signal 5 (error 0.4)
    assert np.allclose(D2[1], X[5] / np.linalg.norm(X[5]))
    # atoms 4 and 5 (parent 2, no signal holds it): from all, the two worst
    assert np.allclose(D2[4], X[1] / np.linalg.norm(X[1]))
    assert np.allclose(D2[5], X[4] / np.linalg.norm(X[4]))


def test_replacement_represents_the_worst_signal_exactly():
    """Property: after a replacement, the worst-represented signal is one atom
    of the dictionary, so one OMP step represents it with no error."""
    rng = np.random.default_rng(3)
    X, D, sup, coef = _random_problem(rng)
    err = np.linalg.norm(ksvd.residual(X, D, sup, coef), axis=1)
    D2, rep = ksvd.replace_unused(D, X, sup, err)
    assert rep == [D.shape[0] - 1]
    j = int(np.argmax(err))
    c = D2 @ X[j]
    a = int(np.argmax(np.abs(c)))
    assert a == rep[0] and np.allclose(c[a] * D2[a], X[j])
