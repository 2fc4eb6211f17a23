"""Counter-based noise keyed by node position.

The value drawn at a node depends only on its (periodically wrapped)
coordinates rounded to 1 mm and on the seed, through the SplitMix64 finaliser
(Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014).  Any numbering of the same nodes therefore sees the same field,
and a node shared by several elements gets one value (the field stays
continuous).
"""

import numpy as np

_M = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def wrap(x, L):
    x = np.asarray(x, dtype=np.float64)
    y = np.mod(x + 0.5 * L, L) - 0.5 * L
    # points within 1 um of +L/2 belong to -L/2
    return np.where(y >= 0.5 * L - 1e-6, y - L, y)


def uniform01(xyz, Lx, Ly, seed):
    """U[0,1) per point from wrapped coordinates rounded to 1 mm."""
    x = wrap(xyz[:, 0], Lx)
    y = wrap(xyz[:, 1], Ly)
    z = np.asarray(xyz[:, 2], dtype=np.float64)
    kx = np.rint(x * 1e3).astype(np.int64).astype(np.uint64)
    ky = np.rint(y * 1e3).astype(np.int64).astype(np.uint64)
    kz = np.rint(z * 1e3).astype(np.int64).astype(np.uint64)
    with np.errstate(over="ignore"):
        h = splitmix64(kz)
        h = splitmix64(h ^ ky)
        h = splitmix64(h ^ kx)
        h = splitmix64(h ^ np.uint64(seed))
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
