"""Pins for the graph and path sampler of the oracle (Def. 1, Alg. 1) on the CPU."""
import itertools
import math

import numpy as np
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
