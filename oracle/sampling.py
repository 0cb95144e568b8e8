"""Tensor sampling: random multipartite graph and path sampling (oracle side).

Def. 1 (Section 3.1): the graph G has L layers (the paper's M), each holding W
waypoints (the paper's N) drawn uniformly over the control box; edges join
every node of layer l to every node of layer l+1, so there are W**L paths.
Alg. 1: draw B index rows I in {0..W-1}^L with replacement and gather the
waypoints C[b, l] = Z[l, I[b, l]].  The paper's randint(1, N) is 1-based;
here indices are 0-based.  Alg. 2 redraws the graph in every loop body; the
planner here redraws it for every CEM iteration k of every replan r.
"""
import numpy as np

from . import philox


def waypoints(seed, r, k, n_layers, n_width, ctrl_dim, u_min, u_max):
    """Z[l, w, j] = u_min + (u_max - u_min) * u01, rounded once to float32.

    The GPU evaluates the same expression as one fused multiply-add in float32;
    the float64 value below is exact for the control limits used here, so its
    single rounding to float32 reproduces the GPU bits."""
    lo = np.float64(np.float32(u_min))
    span = np.float64(np.float32(np.float32(u_max) - np.float32(u_min)))
    words = philox.stream_words(seed, philox.TAG_Z, r, k, np.arange(n_layers),
                                n_width * ctrl_dim)
    f = philox.u01(words)                                   # (L, W*n)
    z = (span * f + lo).astype(np.float32)
    return z.reshape(n_layers, n_width, ctrl_dim)


def path_indices(seed, r, k, n_paths, n_layers, n_width):
    """Alg. 1, first line: I[p, l] uniform in {0..W-1}, with replacement."""
    words = philox.stream_words(seed, philox.TAG_I, r, k, np.arange(n_paths), n_layers)
    return philox.index_of(words, n_width)                  # (P, L) int64


def gather(Z, I):
    """Alg. 1, second line: C[p, l, :] = Z[l, I[p, l], :]."""
    L = Z.shape[0]
    return Z[np.arange(L)[None, :], I, :]                   # (P, L, n)
