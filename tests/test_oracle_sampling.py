"""Pins for the graph and path sampler of the oracle (Def. 1, Alg. 1) on the CPU."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import sampling, philox


def test_waypoints_inside_box_and_float32_exact():
    Z = sampling.waypoints(3, 0, 0, 5, 30, 2, -1.0, 1.0)
    assert Z.shape == (5, 30, 2) and Z.dtype == np.float32
    assert Z.min() >= -1.0 and Z.max() < 1.0
    # value equals lo + span*u01 exactly representable: re-derive with python floats
    words = philox.stream_words(3, philox.TAG_Z, 0, 0, np.arange(5), 60)
    for l in range(5):
        for e in range(60):
            f = (int(words[l, e]) >> 8) / 2 ** 24
            assert float(Z[l, e // 2, e % 2]) == float(np.float32(-1.0 + 2.0 * f))


def test_waypoints_uniform():
    Z = sampling.waypoints(1, 2, 3, 8, 64, 24, -5.0, 5.0).ravel()
    assert stats.kstest((Z + 5.0) / 10.0, "uniform").pvalue > 1e-4


def test_path_indices_valid_and_with_replacement():
    I = sampling.path_indices(0, 0, 0, 4096, 6, 10)
    assert I.shape == (4096, 6)
    assert I.min() == 0 and I.max() == 9
    # each layer's index is uniform and layers are independent
    for l in range(6):
        assert stats.chisquare(np.bincount(I[:, l], minlength=10)).pvalue > 1e-4
    tab = np.zeros((10, 10))
    np.add.at(tab, (I[:, 0], I[:, 1]), 1)
    assert stats.chi2_contingency(tab).pvalue > 1e-4


def test_tiny_graph_enumeration_uniform_paths_and_entropy():
    """All W^L paths appear, each with mass 1/W^L (Section 3.1), and the empirical
    path entropy approaches L log W (App. A.2)."""
    L, W, P = 3, 3, 100_000
    I = sampling.path_indices(17, 0, 0, P, L, W)
    code = I @ (W ** np.arange(L))
    counts = np.bincount(code, minlength=W ** L)
    assert counts.shape[0] == W ** L and np.all(counts > 0)
    assert stats.chisquare(counts).pvalue > 1e-4
    p = counts / counts.sum()
    H = -np.sum(p * np.log(p))
    assert abs(H - L * math.log(W)) < 2e-3


def test_gather_picks_layer_waypoints():
    Z = sampling.waypoints(0, 0, 0, 4, 8, 2, -1, 1)
    I = sampling.path_indices(0, 0, 0, 50, 4, 8)
    C = sampling.gather(Z, I)
    for p in range(50):
        for l in range(4):
            assert np.array_equal(C[p, l], Z[l, I[p, l]])


# ------------------------------------------------------------------ without replacement

@pytest.mark.parametrize("W_, L_", [(2, 1), (2, 4), (3, 3), (5, 2), (4, 4), (7, 2)])
def test_permutation_is_a_bijection_of_all_paths(W_, L_):
    """P = W^L paths without replacement enumerate every path exactly once."""
    D = W_ ** L_
    I = sampling.path_indices_without_replacement(11, 3, 1, D, L_, W_)
    assert I.shape == (D, L_) and I.min() >= 0 and I.max() < W_
    num = (I * (W_ ** np.arange(L_))).sum(axis=1)
    assert sorted(num.tolist()) == list(range(D))


def test_permutation_rounds_are_involutions():
    keys, fkeys = sampling.perm_round_keys(5, 2, 0, 6, 9)
    D = 9 ** 6
    x = [int(v) for v in np.random.default_rng(0).integers(0, D, 500)]
    for K, fk in list(zip(keys, fkeys))[:6]:
        assert sampling.perm_round(sampling.perm_round(x, K, fk, 6, 9), K, fk, 6, 9) == x
    assert len(keys) == sampling.perm_rounds(6, 9) == 2 * 6 * 4


def test_digits_recompose():
    x = [0, 1, 63, 64, 2 ** 40 - 1, 12345678901]
    d = sampling.digits(x, 8, 32)
    assert [int(sum(int(v) * 32 ** l for l, v in enumerate(row))) for row in d] == x


def test_without_replacement_beyond_64_bits():
    """W^L = 64^12 = 2^72 paths: the exact integer arithmetic still yields distinct paths."""
    I = sampling.path_indices_without_replacement(0, 0, 0, 300, 12, 64)
    assert len({tuple(r) for r in I}) == 300 and I.max() < 64


def test_with_replacement_collides_where_without_does_not():
    """At 200 of 4^4 = 256 paths draws with replacement repeat paths (birthday
    bound), draws without replacement never do."""
    Iw = sampling.path_indices(0, 0, 0, 200, 4, 4)
    Io = sampling.path_indices_without_replacement(0, 0, 0, 200, 4, 4)
    assert len({tuple(r) for r in Iw}) < 200
    assert len({tuple(r) for r in Io}) == 200


def test_permutation_is_close_to_uniform():
    """Over many replan indices the first path is uniform over the 8 paths of a
    2^3 graph and the first two form a uniform ordered pair of distinct paths
    (chi-square at the 0.1% level)."""
    from scipy import stats
    n = 1500
    first, pair = [], []
    for r in range(n):
        I = sampling.path_indices_without_replacement(7, r, 0, 2, 3, 2)
        a, b = (int((row * (2 ** np.arange(3))).sum()) for row in I)
        first.append(a)
        pair.append(a * 8 + b)
    c1 = np.bincount(first, minlength=8)
    assert stats.chisquare(c1).pvalue > 1e-3
    c2 = np.bincount(pair, minlength=64).reshape(8, 8)
    assert np.all(np.diag(c2) == 0)
    off = c2[~np.eye(8, dtype=bool)]
    assert stats.chisquare(off).pvalue > 1e-3
