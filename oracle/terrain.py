"""Terrain-following (mapped) hexahedra for the right-hand side (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Section 3 defines the basis through mappings xi(x), eta(x), zeta(x) from each
physical element onto the reference cube.  The paper's runs use box elements,
for which the mapping is affine (``oracle.euler``).  This module takes the
general case for a terrain-following vertical coordinate: the columns keep
their horizontal boxes, and a node at flat height zf (layer edges plus LGL
positions, as in ``oracle.mesh``) over a surface of height zs above the flat
bottom z0 moves to

    z = zf + zs (H - zf) / (H - z0),          H = top of the domain,

so the surface follows the terrain and the top stays flat.

Everything below is the textbook mapped-element machinery, written for any
mapping (nothing assumes the terrain-following form beyond ``physical_z``):

* Jacobian J[a, b] = d x_a / d xi_b at every local node, obtained by applying
  the LGL derivative matrix to the nodal coordinates (discrete metrics);
* physical derivative by the chain rule, d f/d x_a = sum_b (J^-1)[b, a] d f/d xi_b;
* lumped mass w_i w_j w_k det J, assembled as M_G = Z^T m_L (Section 3.1);
* reference state given per unique node (its value at the node's physical
  height) and scattered like the solution.

The sub-grid (horizontal Smagorinsky-Lilly) and absorbing-layer terms of the
model setup follow ``oracle.euler.dissipation`` with physical derivatives, and
the layer is placed by each node's physical height.

Boundary: the top is a rigid lid (the w tendency is removed, as in
``oracle.assembly``).  At the terrain surface the momentum tendency loses its
component along the surface normal n ~ (-dzs/dx, -dzs/dy, 1), with the
horizontal gradient of zs taken element by element and averaged with the
lumped masses over the elements sharing the surface node (a direct stiffness
summation); on flat ground this is the lid rule again.  The paper has no
terrain: this boundary rule is a reading, not the paper's.
"""

import numpy as np

from . import assembly, euler
from .gll import derivative_matrix


def physical_z(mesh, zsG):
    """Physical height of every local node, shape (E, n, n, n).

    zsG: surface height above the flat bottom at every unique node (the same
    value along a column of nodes), scattered to the local nodes with Z."""
    z0, H = mesh.z_edges[0], mesh.z_edges[-1]
    zsL = assembly.scatter(mesh, np.asarray(zsG, dtype=np.float64)[None])[0]
    return mesh.zl + zsL * (H - mesh.zl) / (H - z0)


def reference_derivatives(D, f):
    """(d f/d xi, d f/d eta, d f/d zeta) of local fields (E, k, j, i)."""
    return (np.einsum("im,ekjm->ekji", D, f),
            np.einsum("jm,ekmi->ekji", D, f),
            np.einsum("km,emji->ekji", D, f))


def jacobian(mesh, zp):
    """J[..., a, b] = d x_a / d xi_b (a: x, y, z; b: xi, eta, zeta) and its
    inverse and determinant at every local node."""
    D = derivative_matrix(mesh.N)
    J = np.empty(mesh.local_shape() + (3, 3))
    for a, coord in enumerate((mesh.xl, mesh.yl, zp)):
        for b, d in enumerate(reference_derivatives(D, coord)):
            J[..., a, b] = d
    return J, np.linalg.inv(J), np.linalg.det(J)


def gradient(mesh, Jinv, f):
    """Physical gradient (d/dx, d/dy, d/dz) of local fields by the chain rule,
    in the precision of f (Jinv is expected in the same precision)."""
    D = derivative_matrix(mesh.N).astype(np.asarray(f).dtype)
    r = reference_derivatives(D, f)
    return tuple(sum(Jinv[..., b, a] * r[b] for b in range(3)) for a in range(3))


def dissipation(mesh, qL, phys, Jinv, zp):
    """The sub-grid and absorbing-layer tendencies of ``oracle.euler.dissipation``
    on mapped elements, FP64: the strain rate and the divergence of the stress
    take the physical derivatives (``gradient``), Delta stays the element's
    mean horizontal node spacing (dx + dy)/(2N), and the absorbing layer is
    evaluated at every node's physical height zp."""
    grad = lambda f: gradient(mesh, Jinv, f)
    out = np.zeros_like(qL)
    cs = phys.get("Cs", 0.0)
    if cs > 0.0:
        u, v, w = qL[1], qL[2], qL[3]
        ux, uy, uz = grad(u)
        vx, vy, vz = grad(v)
        wx, wy, wz = grad(w)
        sxx, syy, szz = ux, vy, wz
        sxy, sxz, syz = 0.5 * (uy + vx), 0.5 * (uz + wx), 0.5 * (vz + wy)
        ss = sxx**2 + syy**2 + szz**2 + 2.0 * (sxy**2 + sxz**2 + syz**2)
        delta = (mesh.e_dx + mesh.e_dy) / (2.0 * mesh.N)
        nu = (cs * delta)[:, None, None, None] ** 2 * np.sqrt(2.0 * ss)
        txx, txy, tyy, txz, tyz = (2.0 * nu * a for a in (sxx, sxy, syy, sxz, syz))
        out[1] += grad(txx)[0] + grad(txy)[1]
        out[2] += grad(txy)[0] + grad(tyy)[1]
        out[3] += grad(txz)[0] + grad(tyz)[1]
    gam = phys.get("sponge_gamma", 0.0)
    if gam > 0.0:
        rz = euler.sponge_profile(zp, mesh.z_edges[-1], gam, phys.get("sponge_depth", 4000.0))
        out -= rz[None] * qL
    return out


def element_rhs(mesh, qL, refL, Jinv, phys, dtype=np.float64, zp=None):
    """Strong-form right-hand side of Section 2 on mapped elements.

    The same pointwise terms as ``oracle.euler.element_rhs``, with every
    derivative taken by ``gradient``.  refL: local rho0, theta0, dtheta0dz.
    dtype: float64, or float32 for the reduced-precision variant, as in
    ``oracle.euler.element_rhs``: state, reference, inverse Jacobian, the
    derivatives and the pointwise terms are float32 arrays (p' is the exact
    difference rounded to float32); the caller's assembly stays FP64.
    zp: physical heights of the local nodes, needed when phys enables the
    dissipation (``dissipation``, evaluated in FP64 on the given state).
    Returns R_L, shape (5, E, n, n, n), float64."""
    q64, Jinv64 = np.asarray(qL, dtype=np.float64), np.asarray(Jinv, dtype=np.float64)
    rho0, theta0, dth0 = refL["rho0"], refL["theta0"], refL["dtheta0dz"]
    pp = euler.pressure_perturbation(rho0, theta0, qL[0], qL[4],
                                     phys["R_d"], phys["c_p"], phys["p00"]).astype(dtype)
    qL = np.asarray(qL).astype(dtype)
    rho0, dth0 = np.asarray(rho0).astype(dtype), np.asarray(dth0).astype(dtype)
    Jinv = np.asarray(Jinv).astype(dtype)
    rho_p, u, v, w, th_p = qL
    rho = rho0 + rho_p
    grad = lambda f: gradient(mesh, Jinv, f)
    mx, _, _ = grad(rho * u)
    _, my, _ = grad(rho * v)
    _, _, mz = grad(rho * w)
    ux, uy, uz = grad(u)
    vx, vy, vz = grad(v)
    wx, wy, wz = grad(w)
    px, py, pz = grad(pp)
    tx, ty, tz = grad(th_p)
    f, g = dtype(phys["f"]), dtype(phys["g"])
    R = np.empty_like(qL)
    R[0] = -(mx + my + mz)
    R[1] = -(u * ux + v * uy + w * uz) - px / rho + f * v
    R[2] = -(u * vx + v * vy + w * vz) - py / rho - f * u
    R[3] = -(u * wx + v * wy + w * wz) - pz / rho - (rho_p / rho) * g
    R[4] = -(u * tx + v * ty + w * tz) - w * dth0
    R = R.astype(np.float64)
    if phys.get("Cs", 0.0) > 0.0 or phys.get("sponge_gamma", 0.0) > 0.0:
        R += dissipation(mesh, q64, phys, Jinv64, zp)
    return R


def lumped_mass(mesh, detJ):
    """m_L = w_i w_j w_k det J per local node (flattened) and M_G = Z^T m_L."""
    w = mesh.w
    w3 = w[:, None, None] * w[None, :, None] * w[None, None, :]     # (k, j, i)
    mL = (w3[None] * detJ).reshape(-1)
    return mL, mesh.ZT @ mL


def surface_nodes(mesh):
    """Unique nodes on the flat bottom of the computational mesh."""
    z0, H = mesh.z_edges[0], mesh.z_edges[-1]
    return np.abs(mesh.node_xyz[:, 2] - z0) < 1e-9 * (H - z0)


def top_nodes(mesh):
    z0, H = mesh.z_edges[0], mesh.z_edges[-1]
    return np.abs(mesh.node_xyz[:, 2] - H) < 1e-9 * (H - z0)


def surface_normal(mesh, zsG, Jinv, mL, MG):
    """Unit normal of the terrain at every unique surface node, (3, n_bottom).

    The horizontal gradient of zs is evaluated element by element (chain rule
    on the mapped element: zs does not vary along a column, so this is its
    horizontal derivative), then averaged over the elements sharing the node
    with the lumped masses (direct stiffness summation)."""
    zsL = assembly.scatter(mesh, np.asarray(zsG, dtype=np.float64)[None])[0]
    gx, gy, _ = gradient(mesh, Jinv, zsL)
    acc = assembly.assemble(mesh, np.stack([gx.reshape(-1) * mL, gy.reshape(-1) * mL]))
    sx, sy = acc / MG[None]
    bot = surface_nodes(mesh)
    nx, ny = -sx[bot], -sy[bot]
    nrm = np.sqrt(1.0 + nx * nx + ny * ny)
    return np.stack([nx / nrm, ny / nrm, 1.0 / nrm]), bot


def rhs(mesh, qG, refG, zsG, phys, dtype=np.float64):
    """Global right-hand side on the terrain-following mesh.

    qG: (5, n_dof) state; refG: dict of rho0, theta0, dtheta0dz per unique
    node (at each node's physical height); zsG: surface height per unique node;
    dtype: precision of the element arithmetic (``element_rhs``).
    Scatter, mapped element RHS, mass-weighted gather, boundary rules."""
    zp = physical_z(mesh, zsG)
    _, Jinv, detJ = jacobian(mesh, zp)
    qL = assembly.scatter(mesh, qG)
    refL = {k: assembly.scatter(mesh, np.asarray(refG[k], dtype=np.float64)[None])[0]
            for k in ("rho0", "theta0", "dtheta0dz")}
    RL = element_rhs(mesh, qL, refL, Jinv, phys, dtype, zp)
    mL, MG = lumped_mass(mesh, detJ)
    RG = assembly.assemble(mesh, RL.reshape(5, -1) * mL[None]) / MG[None]
    # top: rigid lid
    RG[3, top_nodes(mesh)] = 0.0
    # terrain surface: remove the normal component of the momentum tendency
    n, bot = surface_normal(mesh, zsG, Jinv, mL, MG)
    Rv = RG[1:4, bot]
    RG[1:4, bot] = Rv - np.sum(Rv * n, axis=0)[None] * n
    return RG


def node_heights(mesh, zsG):
    """Physical height of every unique node (for evaluating the reference)."""
    z0, H = mesh.z_edges[0], mesh.z_edges[-1]
    zf = mesh.node_xyz[:, 2]
    return zf + np.asarray(zsG, dtype=np.float64) * (H - zf) / (H - z0)


def criterion_vorticity(mesh, qL, zsG):
    """Vertical relative vorticity dv/dx - du/dy at every local node of the
    mapped elements (element-local values, as the refinement criterion of
    Section 4.1 reads them), by the chain rule of the mapping."""
    _, Jinv, _ = jacobian(mesh, physical_z(mesh, zsG))
    vx, _, _ = gradient(mesh, Jinv, qL[2])
    _, uy, _ = gradient(mesh, Jinv, qL[1])
    return vx - uy
