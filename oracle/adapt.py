"""One adaptation pass of the column quadtree and the transfer of the solution
onto the adapted mesh (oracle, FP64, test infrastructure only).

Section 4.1 adapts whole columns: a flagged column is split into a 2 x 2
block of columns, and four sibling columns that are all flagged for
coarsening are merged back into their parent.  The paper leaves the mesh
bookkeeping to its mesh library and does not describe how the solution moves
to the new elements; the readings used here are:

Layout (``adapt_columns``)
  1. every column flagged +1 below ``lvl_max`` is split into its four
     children;
  2. 2:1 balance across faces and corners is restored by splitting any leaf
     that touches a leaf two or more levels finer, until none does (the
     unique coarsest balanced refinement of step 1);
  3. four sibling leaves that were all flagged -1 are merged, provided every
     leaf of the balanced layout touching the parent's box is at most one
     level finer than the parent.  All merges are decided on the layout of
     step 2 at once, so the result does not depend on any visiting order.

Solution (``transfer``)
  * an element that exists in both layouts keeps its local values;
  * a child of a split column takes its parent's polynomial at its own nodes
    (interpolation: exact, the polynomial is unchanged);
  * a merged parent takes the discrete L2 projection of its four children:
    the polynomial of order N minimising sum m_n (p(x_n) - q_c(x_n))^2 over
    the children's LGL nodes with their lumped masses m_n (conserves the
    element's sum of m q);
  * the global value at a unique node of the new mesh is the old field at
    that point whenever the node belongs to a kept or split-child element;
    at a node that belongs only to merged parents it is the lumped-mass
    weighted average of their projections.
"""

import numpy as np

from .gll import lagrange_matrix


# ---------------------------------------------------------------- layouts
def _leaf_over(leaves, l, x, y):
    """The leaf containing cell (l, x, y) if that cell is not subdivided."""
    for la in range(l, -1, -1):
        s = l - la
        key = (la, x >> s, y >> s)
        if key in leaves:
            return key
    return None


def _neighbour_cells(l, x, y, nx0, ny0, periodic_x, periodic_y):
    nxl, nyl = nx0 << l, ny0 << l
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            a, b = x + dx, y + dy
            if periodic_x:
                a %= nxl
            elif not 0 <= a < nxl:
                continue
            if periodic_y:
                b %= nyl
            elif not 0 <= b < nyl:
                continue
            yield a, b


def finest_level_map(leaves, nx0, ny0, depth):
    """Level of the leaf covering each cell of the level-``depth`` grid."""
    m = -np.ones((nx0 << depth, ny0 << depth), dtype=np.int64)
    for (l, x, y) in leaves:
        s = 1 << (depth - l)
        m[x * s:(x + 1) * s, y * s:(y + 1) * s] = l
    return m


def ring_max_level(lmap, l, x, y, depth, periodic_x, periodic_y):
    """Largest leaf level among the finest cells bordering the box of cell
    (l, x, y) across its faces and corners."""
    s = 1 << (depth - l)
    nx, ny = lmap.shape
    xs = np.arange(x * s - 1, (x + 1) * s + 1)
    ys = np.arange(y * s - 1, (y + 1) * s + 1)
    best = -1
    for a in xs:
        for b in ys:
            if x * s <= a < (x + 1) * s and y * s <= b < (y + 1) * s:
                continue
            if periodic_x:
                a = a % nx
            elif not 0 <= a < nx:
                continue
            if periodic_y:
                b = b % ny
            elif not 0 <= b < ny:
                continue
            best = max(best, int(lmap[a, b]))
    return best


def is_balanced(leaves, nx0, ny0, periodic_x=True, periodic_y=True):
    """Brute-force 2:1 check on the finest grid: no leaf touches a leaf more
    than one level finer."""
    depth = max(l for l, _, _ in leaves)
    lmap = finest_level_map(leaves, nx0, ny0, depth)
    if (lmap < 0).any():
        return False
    return all(ring_max_level(lmap, l, x, y, depth, periodic_x, periodic_y) <= l + 1
               for (l, x, y) in leaves)


def adapt_columns(columns, adapt_col, nx0, ny0, lvl_max, periodic_x=True, periodic_y=True):
    """New leaf set (a Python set of (level, ix, iy)) after one pass."""
    cols = [tuple(int(t) for t in c) for c in np.asarray(columns).reshape(-1, 3)]
    flags = np.asarray(adapt_col).reshape(-1)
    if len(flags) != len(cols):
        raise ValueError("one flag per column")
    # 1. split
    leaves = set()
    for (l, x, y), f in zip(cols, flags):
        if f == 1 and l < lvl_max:
            leaves.update((l + 1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1))
        else:
            leaves.add((l, x, y))
    # 2. balance by splitting leaves that touch leaves two levels finer
    while True:
        split = set()
        for (l, x, y) in leaves:
            for a, b in _neighbour_cells(l, x, y, nx0, ny0, periodic_x, periodic_y):
                nb = _leaf_over(leaves, l, a, b)
                if nb is not None and nb[0] < l - 1:
                    split.add(nb)
        if not split:
            break
        for (l, x, y) in split:
            leaves.discard((l, x, y))
            leaves.update((l + 1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1))
    # 3. merge complete flagged families if the parent stays balanced
    coarsen = {c for c, f in zip(cols, flags) if f == -1 and c[0] > 0}
    depth = max(l for l, _, _ in leaves)
    lmap = finest_level_map(leaves, nx0, ny0, depth)
    parents = {(l - 1, x >> 1, y >> 1) for (l, x, y) in coarsen}
    merged = []
    for (l, x, y) in sorted(parents):
        kids = [(l + 1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1)]
        if not all(k in coarsen and k in leaves for k in kids):
            continue
        if ring_max_level(lmap, l, x, y, depth, periodic_x, periodic_y) <= l + 1:
            merged.append(((l, x, y), kids))
    for p, kids in merged:
        leaves.difference_update(kids)
        leaves.add(p)
    return leaves


# ---------------------------------------------------------------- transfer
def classify(old_columns, new_columns):
    """For each new column: ('same', [old]), ('child', [old parent]) or
    ('parent', [four old children, a along x then b along y])."""
    idx = {tuple(int(t) for t in c): i for i, c in enumerate(np.asarray(old_columns).reshape(-1, 3))}
    out = []
    for c in np.asarray(new_columns).reshape(-1, 3):
        l, x, y = (int(t) for t in c)
        if (l, x, y) in idx:
            out.append(("same", [idx[(l, x, y)]]))
        elif l > 0 and (l - 1, x >> 1, y >> 1) in idx:
            out.append(("child", [idx[(l - 1, x >> 1, y >> 1)]]))
        else:
            kids = [(l + 1, 2 * x + a, 2 * y + b) for b in (0, 1) for a in (0, 1)]
            if not all(k in idx for k in kids):
                raise ValueError("column %s has no counterpart one level apart" % ((l, x, y),))
            out.append(("parent", [idx[k] for k in kids]))
    return out


def _ref_coords(mesh_from, col, xs, ys):
    """Reference coordinates in [-1, 1] of points inside column ``col``."""
    sx = 2.0 * (xs - mesh_from.col_x0[col]) / mesh_from.col_wx[col] - 1.0
    sy = 2.0 * (ys - mesh_from.col_y0[col]) / mesh_from.col_wy[col] - 1.0
    return sx, sy


def element_transfer(old, new, qL_old):
    """Element-local values on the new mesh, shape (F, E_new, n, n, n)."""
    n, nz = new.np1, new.n_z
    kinds = classify(old.columns, new.columns)
    F = qL_old.shape[0]
    out = np.zeros((F, new.n_elem, n, n, n))
    for c, (kind, src) in enumerate(kinds):
        for layer in range(nz):
            e = c * nz + layer
            if kind == "same":
                out[:, e] = qL_old[:, src[0] * nz + layer]
            elif kind == "child":
                ep = src[0] * nz + layer
                sx, _ = _ref_coords(old, src[0], new.xl[e, 0, 0, :], new.yl[e, 0, 0, :])
                _, sy = _ref_coords(old, src[0], new.xl[e, 0, :, 0], new.yl[e, 0, :, 0])
                Lx = lagrange_matrix(old.xi, sx)      # (i, m)
                Ly = lagrange_matrix(old.xi, sy)      # (j, p)
                out[:, e] = np.einsum("im,jp,fkpm->fkji", Lx, Ly, qL_old[:, ep])
            else:
                # discrete L2 projection over the children's LGL nodes
                rows, rhs, wts = [], [], []
                for ch in src:
                    ec = ch * nz + layer
                    sx, sy = _ref_coords(new, c, old.xl[ec].reshape(-1), old.yl[ec].reshape(-1))
                    sz = 2.0 * (old.zl[ec].reshape(-1) - new.e_z0[e]) / new.e_dz[e] - 1.0
                    A = (lagrange_matrix(new.xi, sz)[:, :, None, None]
                         * lagrange_matrix(new.xi, sy)[:, None, :, None]
                         * lagrange_matrix(new.xi, sx)[:, None, None, :]).reshape(sx.size, -1)
                    rows.append(A)
                    rhs.append(qL_old[:, ec].reshape(F, -1).T)
                    wts.append(old.mL.reshape(old.n_elem, -1)[ec])
                A = np.concatenate(rows)
                B = np.concatenate(rhs)
                sw = np.sqrt(np.concatenate(wts))
                coef, *_ = np.linalg.lstsq(sw[:, None] * A, sw[:, None] * B, rcond=None)
                out[:, e] = coef.T.reshape(F, n, n, n)
    return out, kinds


def transfer(old, new, q_old):
    """Global state on the new mesh from the global state on the old one.

    old, new : OracleMesh with the same order, vertical layers and domain.
    q_old    : (F, old.n_dof) in the old mesh's unique-node order.
    Returns (F, new.n_dof) in the new mesh's unique-node order.
    """
    q_old = np.atleast_2d(q_old)
    F = q_old.shape[0]
    qL_old = np.stack([old.Z @ q_old[f] for f in range(F)]).reshape((F,) + old.local_shape())
    qt, kinds = element_transfer(old, new, qL_old)
    qt = qt.reshape(F, -1)
    n3 = new.np1 ** 3
    kind_of_elem = np.repeat(np.array([k for k, _ in kinds]), new.n_z)
    Zc = new.Z.tocoo()
    unit = ~new.hanging[Zc.row]
    loc, u = Zc.row[unit], Zc.col[unit]
    exact = np.isin(kind_of_elem[loc // n3], ("same", "child"))
    out = np.full((F, new.n_dof), np.nan)
    have = np.zeros(new.n_dof, dtype=bool)
    # nodes of kept or split-child elements: the old field at that point
    for l, g in zip(loc[exact], u[exact]):
        if not have[g]:
            out[:, g] = qt[:, l]
            have[g] = True
    # nodes of merged parents only: mass-weighted average of the projections
    num = np.zeros((F, new.n_dof))
    den = np.zeros(new.n_dof)
    proj = ~exact
    np.add.at(den, u[proj], new.mL[loc[proj]])
    for f in range(F):
        np.add.at(num[f], u[proj], new.mL[loc[proj]] * qt[f, loc[proj]])
    rest = ~have
    out[:, rest] = num[:, rest] / den[rest]
    return out
