"""Shared test helpers: build the oracle and GPU sides of one case and match
their unique-node numberings by position (never by shared code)."""

import numpy as np

from oracle.mesh import OracleMesh
from synth import cases


def oracle_mesh(case):
    return OracleMesh(case["N"], case["nx0"], case["ny0"], case["Lx"], case["Ly"],
                      case["z_edges"], case["columns"], case["periodic_x"], case["periodic_y"])


def _keys(xyz, case, q=1e-3):
    x = xyz[:, 0].copy()
    y = xyz[:, 1].copy()
    if case["periodic_x"]:
        L = case["Lx"]
        x = np.mod(x + 0.5 * L, L) - 0.5 * L
        x = np.where(x >= 0.5 * L - 1e-6, x - L, x)
    if case["periodic_y"]:
        L = case["Ly"]
        y = np.mod(y + 0.5 * L, L) - 0.5 * L
        y = np.where(y >= 0.5 * L - 1e-6, y - L, y)
    return np.stack([np.rint(x / q), np.rint(y / q), np.rint(xyz[:, 2] / q)], axis=1).astype(np.int64)


def match(a_xyz, b_xyz, case):
    """perm with b_xyz[i] == a_xyz[perm[i]] (bijective, checked)."""
    ka, kb = _keys(a_xyz, case), _keys(b_xyz, case)
    if ka.shape != kb.shape:
        raise AssertionError(f"node counts differ: {ka.shape[0]} vs {kb.shape[0]}")
    ia = np.lexsort(ka.T[::-1])
    ib = np.lexsort(kb.T[::-1])
    if not np.array_equal(ka[ia], kb[ib]):
        raise AssertionError("node sets differ")
    perm = np.empty(ka.shape[0], dtype=np.int64)
    perm[ib] = ia
    return perm


def oracle_reference_local(case, om):
    bg = cases.reference_state(case, om.zl)
    return dict(rho0=bg["rho0"], theta0=bg["theta0"], dtheta0dz=bg["dtheta0dz"])
