"""Direct stiffness summation with hanging nodes (FP64).

Section 3.1: the global (continuous) solution is assembled from the local
element values by direct stiffness summation (DSS).  With hanging nodes the
local values at a hanging node are passed to the non-hanging nodes through
the interpolation that defines it, the mass matrix is assembled the same way,
and the global solution is interpolated back onto the hanging nodes.  In
matrix form, with Z the local-from-global interpolation of ``oracle.mesh``:

    scatter  : q_L = Z q_G
    gather   : R_G = (Z^T (m_L * R_L)) / M_G,   M_G = Z^T m_L

A rigid lid at the bottom and top removes the vertical-velocity tendency at
those nodes (no-flux lids of the workloads).
"""

import numpy as np


def scatter(mesh, qG):
    """q_L = Z q_G for every field; returns shape (F, E, n, n, n)."""
    qG = np.atleast_2d(qG)
    out = np.stack([mesh.Z @ qG[f] for f in range(qG.shape[0])])
    return out.reshape((qG.shape[0],) + mesh.local_shape())


def assemble(mesh, cL):
    """Z^T c_L for already mass-weighted local contributions (F, n_loc)."""
    cL = cL.reshape(cL.shape[0], -1)
    return np.stack([mesh.ZT @ cL[f] for f in range(cL.shape[0])])


def gather(mesh, RL, lid_field=3):
    """R_G = Z^T(m_L R_L) / M_G, then R_w = 0 on the lid nodes."""
    RL = RL.reshape(RL.shape[0], -1)
    acc = assemble(mesh, RL * mesh.mL[None, :])
    RG = acc / mesh.MG[None, :]
    if lid_field is not None and RG.shape[0] > lid_field:
        RG[lid_field, mesh.lid] = 0.0
    return RG


def rhs(mesh, qG, ref_local, phys, dtype=np.float64):
    """Global right-hand side: scatter, element RHS, gather (Sections 2-3).
    dtype=float32 evaluates the element right-hand side in float32 (the
    reduced-precision variant); scatter and gather stay FP64."""
    from .euler import element_rhs
    qL = scatter(mesh, qG)
    RL = element_rhs(mesh, qL, ref_local["rho0"], ref_local["theta0"],
                     ref_local["dtheta0dz"], phys, dtype=dtype)
    return gather(mesh, RL)
