"""Refinement / coarsening flags (Section 4.1).

Each element e has a level lvl(e) in [0, lvl_max] and a criterion value C at
each of its nodes.  With per-level thresholds threshold(1..lvl_max):

* refine (+1)  if some node has C > threshold(lvl(e)+1) and lvl(e) < lvl_max;
* coarsen (-1) if every node has C <= threshold(lvl(e)) and lvl(e) > 0
  (level 0 has no coarsening threshold: it is the largest element size);
* otherwise keep (0).

A level changes by at most one per adaptation pass (the paper's remark), so
the flag is in {-1, 0, +1}.  The oracle follows the prose rule rather than
the printed algorithm, whose inner test indexes an undefined threshold and
lets a later node overwrite an earlier decision.

Refinement acts on whole columns (Section 4.1, refining an element): a
column is refined when any of its elements is flagged +1; four sibling
columns sharing a corner are merged only if every element of all four is
flagged -1 (coarsening an element).

``thr`` below is 0-based: thr[l-1] = threshold(l).
"""

import numpy as np


def criterion_speed(q_local):
    """Velocity magnitude |u| at every local node; q_local (5, E, ...)."""
    u, v, w = q_local[1], q_local[2], q_local[3]
    return np.sqrt(u * u + v * v + w * w)


def criterion_vorticity(mesh, q_local):
    """Vertical relative vorticity dv/dx - du/dy from element-local
    derivatives (values of the node belonging to the element)."""
    from .gll import derivative_matrix
    from .euler import local_derivatives
    D = derivative_matrix(mesh.N)
    vx, _, _ = local_derivatives(D, q_local[2], mesh.e_dx, mesh.e_dy, mesh.e_dz)
    _, uy, _ = local_derivatives(D, q_local[1], mesh.e_dx, mesh.e_dy, mesh.e_dz)
    return vx - uy


def element_flags(C, lvl, thr, lvl_max):
    """adapt(e) from per-node criterion values C (E, n_nodes)."""
    C = np.asarray(C).reshape(len(lvl), -1)
    cmax = C.max(axis=1)
    lvl = np.asarray(lvl)
    thr = np.asarray(thr, dtype=np.float64)
    if np.any(np.diff(thr) < 0):
        raise ValueError("thresholds must be non-decreasing")
    out = np.zeros(len(lvl), dtype=np.int8)
    for e in range(len(lvl)):
        L = int(lvl[e])
        if L < lvl_max and cmax[e] > thr[L]:
            out[e] = 1
        elif L > 0 and cmax[e] <= thr[L - 1]:
            out[e] = -1
    return out


def column_flags(elem_flags, columns, n_z):
    """Per-column flag with the whole-column and four-sibling rules."""
    ef = np.asarray(elem_flags).reshape(-1, n_z)
    ncol = ef.shape[0]
    refine = (ef == 1).any(axis=1)
    allc = (ef == -1).all(axis=1)
    cols = np.asarray(columns)
    index = {(int(l), int(x), int(y)): c for c, (l, x, y) in enumerate(cols)}
    out = np.zeros(ncol, dtype=np.int8)
    for c in range(ncol):
        l, x, y = (int(t) for t in cols[c])
        if refine[c]:
            out[c] = 1
            continue
        if l == 0 or not allc[c]:
            continue
        bx, by = x - (x & 1), y - (y & 1)
        sib = [index.get((l, bx + dx, by + dy)) for dx in (0, 1) for dy in (0, 1)]
        if all(s is not None and allc[s] and not refine[s] for s in sib):
            out[c] = -1
    return out
