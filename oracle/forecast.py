"""Refinement forecaster, mesh side (oracle, FP64; test infrastructure only).

The paper's criterion (Section 4.1) thresholds a field at an element's nodes
when the mesh is adapted.  The forecaster predicts the decision a few
adaptation intervals ahead from per-element features; its flags are merged
with the criterion's so that the criterion overrides every refinement the
forecaster misses.  Definitions written out here:

features (per element e, element-local values and derivatives, zeta =
dv/dx - du/dy, u_h = (u, v); over terrain-following coordinates every
derivative is the physical one, by the chain rule of the mapping as in
``oracle.terrain``):
   0 level              1 max|zeta|            2 mean zeta
   3 max|u_h|           4 max|w|               5 max theta'
   6 min theta'         7 max|grad p'|         8 max|grad theta'|
   9 max|div u|        10 max rho' - min rho'
  11 largest max|zeta| and 12 largest max|u_h| over the same-layer elements
     of the columns that share a unique node with e's column
  13 max|u_h| - the same for the previous state
  14 max|zeta| - the same for the previous state
  15 the criterion's element flag
  each multiplied by a given scale.
dem(e): the largest level l in 1..lvl_max whose threshold the criterion's
  element maximum exceeds (0 if none): the level the criterion asks for.
label(e): clip(D - level(e), -1, 1) + 1 with D the dem, at a later time, of
  the element covering e's footprint (or the largest over the later elements
  inside it).
forecast flags: class argmax of the logits (first maximum), clamped to the
  level range, then refine if the forecast or the criterion refines, coarsen
  only if both coarsen; columns by the whole-column and sibling rules.
"""

import numpy as np

from . import terrain
from .amr import column_flags
from .euler import local_derivatives, pressure_perturbation
from .gll import derivative_matrix


def element_stats(mesh, qL, ref_local, phys, criterion, zsG=None):
    """Raw per-element quantities of one state: dict of arrays (E,).

    ref_local: rho0, theta0 at the local nodes (over terrain, at every node's
    physical height); zsG: surface height per unique node, or None for box
    elements."""
    rp, u, v, w, tp = qL
    if zsG is None:
        D = derivative_matrix(mesh.N)
        d = lambda f: local_derivatives(D, f, mesh.e_dx, mesh.e_dy, mesh.e_dz)
    else:
        _, Jinv, _ = terrain.jacobian(mesh, terrain.physical_z(mesh, zsG))
        d = lambda f: terrain.gradient(mesh, Jinv, f)
    pp = pressure_perturbation(ref_local["rho0"], ref_local["theta0"], rp, tp,
                               phys["R_d"], phys["c_p"], phys["p00"])
    ux, uy, uz = d(u)
    vx, vy, vz = d(v)
    wx, wy, wz = d(w)
    px, py, pz = d(pp)
    tx, ty, tz = d(tp)
    zeta = vx - uy
    E = mesh.n_elem
    flat = lambda a: a.reshape(E, -1)
    out = dict(
        zabs=flat(np.abs(zeta)).max(1), zmean=flat(zeta).mean(1),
        uh=flat(np.sqrt(u * u + v * v)).max(1), w=flat(np.abs(w)).max(1),
        tmax=flat(tp).max(1), tmin=flat(tp).min(1),
        gp=flat(np.sqrt(px * px + py * py + pz * pz)).max(1),
        gt=flat(np.sqrt(tx * tx + ty * ty + tz * tz)).max(1),
        div=flat(np.abs(ux + vy + wz)).max(1),
        rrange=flat(rp).max(1) - flat(rp).min(1))
    crit = np.sqrt(u * u + v * v + w * w) if criterion == 0 else zeta
    out["crit"] = flat(crit).max(1)
    return out


def neighbour_elements(mesh):
    """For every element, the same-layer elements of other columns that
    share a unique (non-hanging) node with it."""
    n3 = mesh.np1 ** 3
    Zc = mesh.Z.tocoo()
    unit = ~mesh.hanging[Zc.row]
    loc, u = Zc.row[unit], Zc.col[unit]
    elem = loc // n3
    owners = {}
    for e, g in zip(elem, u):
        owners.setdefault(int(g), set()).add(int(e))
    nb = [set() for _ in range(mesh.n_elem)]
    for es in owners.values():
        for e in es:
            nb[e].update(es)
    col = mesh.e_col
    lay = mesh.e_layer
    return [sorted(x for x in nb[e] if col[x] != col[e] and lay[x] == lay[e])
            for e in range(mesh.n_elem)]


def features(mesh, qL, qL_prev, plain_elem, ref_local, phys, criterion, thr, lvl_max, scale,
             zsG=None):
    """(features (E, 16) FP64 already scaled, dem (E,) int); zsG as in
    ``element_stats``."""
    s = element_stats(mesh, qL, ref_local, phys, criterion, zsG)
    sp = element_stats(mesh, qL_prev, ref_local, phys, criterion, zsG)
    E = mesh.n_elem
    F = np.zeros((E, 16))
    F[:, 0] = mesh.e_level
    F[:, 1] = s["zabs"]
    F[:, 2] = s["zmean"]
    F[:, 3] = s["uh"]
    F[:, 4] = s["w"]
    F[:, 5] = s["tmax"]
    F[:, 6] = s["tmin"]
    F[:, 7] = s["gp"]
    F[:, 8] = s["gt"]
    F[:, 9] = s["div"]
    F[:, 10] = s["rrange"]
    for e, nbs in enumerate(neighbour_elements(mesh)):
        F[e, 11] = max([s["zabs"][x] for x in nbs], default=0.0)
        F[e, 12] = max([s["uh"][x] for x in nbs], default=0.0)
    F[:, 13] = s["uh"] - sp["uh"]
    F[:, 14] = s["zabs"] - sp["zabs"]
    F[:, 15] = np.asarray(plain_elem)
    thr = np.asarray(thr, dtype=np.float64)
    dem = np.zeros(E, dtype=np.int64)
    for l in range(1, lvl_max + 1):
        dem[s["crit"] > thr[l - 1]] = l
    return F * np.asarray(scale, dtype=np.float64)[None, :], dem


def forecast_flags(logits, plain_elem, levels, lvl_max, columns, n_z):
    cls = np.argmax(np.asarray(logits), axis=1)
    f = cls - 1
    lv = np.asarray(levels)
    f = np.where((f == 1) & (lv >= lvl_max), 0, f)
    f = np.where((f == -1) & (lv == 0), 0, f)
    p = np.asarray(plain_elem)
    e = np.where((p == 1) | (f == 1), 1, np.where((p == -1) & (f == -1), -1, 0)).astype(np.int8)
    return e, column_flags(e, columns, n_z)


def labels(columns_at, columns_later, dem_later, n_z):
    """Training classes of the elements of layout ``columns_at``."""
    later = {tuple(int(t) for t in c): i for i, c in enumerate(np.asarray(columns_later))}
    dem_later = np.asarray(dem_later).reshape(-1, n_z)
    out = []
    for (l, x, y) in (tuple(int(t) for t in c) for c in np.asarray(columns_at)):
        src = None
        for a in range(l, -1, -1):
            key = (a, x >> (l - a), y >> (l - a))
            if key in later:
                src = dem_later[later[key]]
                break
        if src is None:
            inside = [i for (L, X, Y), i in later.items()
                      if L > l and (X >> (L - l)) == x and (Y >> (L - l)) == y]
            src = dem_later[inside].max(axis=0)
        out.append(np.clip(src - l, -1, 1) + 1)
    return np.concatenate(out).astype(np.int8)
