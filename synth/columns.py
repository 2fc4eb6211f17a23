"""Column layouts for the horizontal quadtree (inputs only).

A layout is an int array (n_col, 3) of (level, ix, iy): a leaf column at
``level`` covering cell (ix, iy) of the nx0*2^level x ny0*2^level grid.
Layouts are returned in Morton (Z-curve) order of their finest-level anchor,
so that columns that are close in space are close in the list.
"""

import numpy as np


def _morton(ix, iy, bits=20):
    key = 0
    for b in range(bits):
        key |= ((ix >> b) & 1) << (2 * b)
        key |= ((iy >> b) & 1) << (2 * b + 1)
    return key


def morton_sort(cols, max_level):
    cols = np.asarray(cols, dtype=np.int64).reshape(-1, 3)
    keys = [_morton(int(x) << (max_level - int(l)), int(y) << (max_level - int(l)))
            for l, x, y in cols]
    order = np.argsort(np.asarray(keys, dtype=np.int64), kind="stable")
    return cols[order]


def uniform(nx0, ny0):
    ix, iy = np.meshgrid(np.arange(nx0), np.arange(ny0), indexing="ij")
    cols = np.stack([np.zeros(ix.size, np.int64), ix.ravel(), iy.ravel()], axis=1)
    return morton_sort(cols, 0)


def _neighbours(l, x, y, nxl, nyl, periodic):
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            a, b = x + dx, y + dy
            if periodic:
                a %= nxl
                b %= nyl
            elif not (0 <= a < nxl and 0 <= b < nyl):
                continue
            yield a, b


def refine_to_target(nx0, ny0, target_level, max_level, periodic=True):
    """Refine from the uniform level-0 layout until every column reaches
    ``target_level(l, ix, iy)`` (capped at max_level), then enforce 2:1
    balance across faces and corners by refining coarse neighbours."""
    leaves = {(0, x, y) for x in range(nx0) for y in range(ny0)}
    for _ in range(max_level):
        nxt = set()
        for (l, x, y) in leaves:
            if l < max_level and target_level(l, x, y) > l:
                nxt.update({(l + 1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1)})
            else:
                nxt.add((l, x, y))
        leaves = nxt
    # 2:1 balance (face + corner): a leaf may not touch a leaf two levels finer
    changed = True
    while changed:
        changed = False
        level_of = {}
        for (l, x, y) in leaves:
            # map every finest-level cell to its leaf level
            s = 1 << (max_level - l)
            for a in range(s):
                for b in range(s):
                    level_of[(x * s + a, y * s + b)] = l
        nxf, nyf = nx0 << max_level, ny0 << max_level
        to_refine = set()
        for (l, x, y) in leaves:
            s = 1 << (max_level - l)
            # finest-level cells just outside this leaf
            ring = []
            for a in range(-1, s + 1):
                ring.append((x * s + a, y * s - 1))
                ring.append((x * s + a, y * s + s))
            for b in range(0, s):
                ring.append((x * s - 1, y * s + b))
                ring.append((x * s + s, y * s + b))
            for (a, b) in ring:
                if periodic:
                    a %= nxf
                    b %= nyf
                elif not (0 <= a < nxf and 0 <= b < nyf):
                    continue
                if level_of[(a, b)] > l + 1:
                    to_refine.add((l, x, y))
                    break
        if to_refine:
            changed = True
            for (l, x, y) in to_refine:
                leaves.remove((l, x, y))
                leaves.update({(l + 1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1)})
    cols = np.array(sorted(leaves), dtype=np.int64)
    return morton_sort(cols, max_level)


def refine_where(nx0, ny0, Lx, Ly, max_level, predicate, periodic=True, samples=9):
    """Refine columns (repeatedly) where ``predicate(x, y, level) -> bool
    array`` holds at any of samples x samples points of the column (edges
    included); ``level`` is the column's current level."""
    def target(l, ix, iy):
        wx = Lx / (nx0 * 2**l)
        wy = Ly / (ny0 * 2**l)
        s = np.linspace(0.0, 1.0, samples)
        X = -0.5 * Lx + (ix + s[:, None]) * wx + 0 * s[None, :]
        Y = -0.5 * Ly + (iy + s[None, :]) * wy + 0 * s[:, None]
        return l + 1 if np.any(predicate(X.ravel(), Y.ravel(), l)) else l
    return refine_to_target(nx0, ny0, target, max_level, periodic)
