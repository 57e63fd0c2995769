"""Keyed standard-normal upstream weights.

A weight is a pure function of (seed, tag, row, col), so any party can
evaluate the weight of one matrix entry without knowing the whole sparsity
pattern.  Construction: SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) hashes the key into two 53-bit
uniforms, and the Box-Muller transform turns them into one N(0, 1) sample.
"""

import numpy as np

_GOLD = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

TAG_D = 1
TAG_M = 2
TAG_G = 3


def _splitmix(x):
    x = (x + _GOLD).astype(np.uint64)
    z = x
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def keyed_normal(seed, tag, row, col):
    """N(0,1) samples keyed by (seed, tag, row, col); row/col are int arrays."""
    with np.errstate(over="ignore"):
        row = np.asarray(row, dtype=np.int64).astype(np.uint64)
        col = np.asarray(col, dtype=np.int64).astype(np.uint64)
        k = _splitmix(np.full(row.shape, (np.uint64(seed) << np.uint64(8)) ^ np.uint64(tag), dtype=np.uint64))
        k = _splitmix(k ^ row)
        k = _splitmix(k ^ col)
        h1 = _splitmix(k)
        h2 = _splitmix(h1)
    u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)  # (0, 1]
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)  # [0, 1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def upstream_weights(seed, D_rows, D_cols, M_rows, M_cols, n_slave_nodes):
    """Weights on the nonzeros of D, of M and on every slave node (gap)."""
    wD = keyed_normal(seed, TAG_D, D_rows, D_cols)
    wM = keyed_normal(seed, TAG_M, M_rows, M_cols)
    idx = np.arange(n_slave_nodes)
    wg = keyed_normal(seed, TAG_G, idx, np.zeros_like(idx))
    return wD, wM, wg
