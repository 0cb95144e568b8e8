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


# ---------------------------------------------------------------- without replacement
# Section 3.2 names sampling paths without replacement as the more diverse but
# costlier variant.  Here path p (0 <= p < P <= W**L) is the image of p under a
# keyed permutation of the W**L path numbers, so distinct p give distinct paths.
# The permutation is the swap-or-not shuffle of Hoang, Morris and Rogaway
# (CRYPTO 2012): each round i has a key K_i in [0, W**L) and a bit function F_i;
# x is replaced by x' = (K_i - x) mod W**L when F_i(max(x, x')) = 1.  Path
# number x names the layer indices by its base-W digits, layer l being digit l
# (least significant first).  Keys and bit functions come from Philox stream 4.
# Python integers carry the modular arithmetic exactly at any W**L.

def perm_rounds(n_layers, n_width):
    """2 L ceil(log2 W) rounds (at least 2 L)."""
    bits = max(1, int(n_width - 1).bit_length())
    return 2 * n_layers * bits


def perm_round_keys(seed, r, k, n_layers, n_width):
    """Per round: the key K_i (a Python int below W**L) and the two words of the
    bit function's Philox key."""
    R = perm_rounds(n_layers, n_width)
    groups = (n_layers + 3) // 4
    k0, k1 = philox.key_of(seed)
    c3 = (philox.TAG_PERM << 16) | (int(k) & 0xFFFF)
    keys, fkeys = [], []
    for i in range(R):
        K = 0
        for l in range(n_layers):
            w = philox.philox4x32_10(i, l // 4, int(r) & 0xFFFFFFFF, c3, k0, k1)[l % 4]
            K += int(philox.index_of(w, n_width)) * n_width ** l
        w = philox.philox4x32_10(i, groups, int(r) & 0xFFFFFFFF, c3, k0, k1)
        keys.append(K)
        fkeys.append((int(w[0]), int(w[1])))
    return keys, fkeys


def digits(x, n_layers, n_width):
    """Base-W digits of the path numbers x (least significant first): (len(x), L) int64."""
    out = np.zeros((len(x), n_layers), dtype=np.int64)
    for i, v in enumerate(x):
        v = int(v)
        for l in range(n_layers):
            v, out[i, l] = divmod(v, n_width)
    return out


def perm_bit(x, fkey, n_layers, n_width):
    """F(x): bit 0 of Philox word 0 with key fkey and the digits of x packed as
    bytes (digit l in byte l % 4 of counter word l // 4)."""
    d = digits(x, n_layers, n_width)
    words = np.zeros((len(x), 4), dtype=np.uint64)
    for l in range(n_layers):
        words[:, l // 4] |= d[:, l].astype(np.uint64) << np.uint64(8 * (l % 4))
    w0 = philox.philox4x32_10(words[:, 0], words[:, 1], words[:, 2], words[:, 3], fkey[0], fkey[1])[0]
    return (w0 & 1).astype(bool)


def perm_round(x, K, fkey, n_layers, n_width):
    """One swap-or-not round on a list of path numbers (an involution)."""
    D = n_width ** n_layers
    xp = [(K - v) % D for v in x]
    hi = [max(a, b) for a, b in zip(x, xp)]
    flip = perm_bit(hi, fkey, n_layers, n_width)
    return [b if f else a for a, b, f in zip(x, xp, flip)]


def path_indices_without_replacement(seed, r, k, n_paths, n_layers, n_width):
    """I[p, l] = digit l of pi(p): P distinct paths of the W**L."""
    if n_paths > n_width ** n_layers:
        raise ValueError("more paths requested than the graph holds")
    keys, fkeys = perm_round_keys(seed, r, k, n_layers, n_width)
    x = list(range(n_paths))
    for K, fk in zip(keys, fkeys):
        x = perm_round(x, K, fk, n_layers, n_width)
    return digits(x, n_layers, n_width)
