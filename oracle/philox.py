"""Philox4x32-10 counter-based generator (oracle side).

Written from the definition in Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11, Section 3 (Philox-4x32, 10 rounds):
each round multiplies counter words 0 and 2 by two fixed 32-bit constants,
xors the high halves with the other counter words and the round key, and
permutes; the two key words are bumped by the Weyl constants (golden ratio and
sqrt(3)-1 in 32-bit fixed point) between rounds.

Pinned by tests against an independent implementation (the header-only
rocRAND engine) and by uniformity statistics.

Stream layout used by the planner (the paper draws with JAX's RNG and fixes
no layout; this one is shared with the GPU path by specification only):
  key      = (seed mod 2^32, seed div 2^32)
  counter  = (block, item, replan index r, (tag << 16) | iteration k)
  tag 1 (graph waypoints Z): item = layer l; element w*n + j
  tag 2 (path indices I):    item = tensor path p; element l
  tag 3 (local noise eps):   item = local sample g; element j*ceil(T/4)*4 + t
  tag 4 (path permutation):  block = round i, item = digit group g (g < ceil(L/4):
                             key digits 4g..4g+3, one per word; g = ceil(L/4):
                             words 0, 1 are the round's bit-function key)
  element e lives in word e % 4 of block e // 4.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

TAG_Z, TAG_I, TAG_EPS, TAG_PERM = 1, 2, 3, 4


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Apply Philox4x32-10 to broadcastable uint32 counter words; returns 4 uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in np.broadcast_arrays(c0, c1, c2, c3))
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def key_of(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def stream_words(seed, tag, r, k, item, n_elem):
    """Words 0..n_elem-1 of the stream (tag, r, k) for every item in `item`.

    Returns uint32 array of shape (len(item), n_elem)."""
    item = np.asarray(item, dtype=np.uint64).reshape(-1, 1)
    n_blocks = (n_elem + 3) // 4
    blk = np.arange(n_blocks, dtype=np.uint64).reshape(1, -1)
    c3 = ((int(tag) & 0xFFFF) << 16) | (int(k) & 0xFFFF)
    k0, k1 = key_of(seed)
    w = philox4x32_10(blk, item, np.uint64(int(r) & 0xFFFFFFFF), np.uint64(c3), k0, k1)
    words = np.stack(w, axis=-1).reshape(item.shape[0], n_blocks * 4)
    return words[:, :n_elem]


def u01(word):
    """Uniform in [0,1): top 24 bits times 2^-24 (exact in float32 and float64)."""
    return (np.asarray(word, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -24


def index_of(word, width):
    """Map a 32-bit word to {0..width-1} by the high half of word*width."""
    return ((np.asarray(word, dtype=np.uint64) * np.uint64(width)) >> _S32).astype(np.int64)


def box_muller(w_a, w_b):
    """Two standard normals from two words (Box and Muller, 1958).

    u1 = (top 24 bits + 1) * 2^-24 lies in (0, 1], so the log is finite."""
    u1 = ((np.asarray(w_a, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) + 1.0) * 2.0 ** -24
    u2 = u01(w_b)
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)
