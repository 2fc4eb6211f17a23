"""Pointwise thermodynamics and strong-form element right-hand side (FP64).

Section 2 writes the dry compressible Euler equations in non-conservative
form for (rho, u, theta), closes them with the ideal-gas law and the Exner
function pi = (p/p0)^(R_d/c_p), splits rho, theta and p into a hydrostatic
reference state depending on z only plus a perturbation, and arrives at the
perturbation system (eqs. mass_split, mom_split, ent_split):

    d rho'/dt  = - div((rho0 + rho') u)
    d u/dt     = - (u . grad) u - grad p' / rho + (rho'/rho) g k,  k = (0,0,-1)
    d theta'/dt= - u . grad theta0 - u . grad theta'

with rho = rho0 + rho'.  The f-plane Coriolis terms (+f v, -f u) are added
to the horizontal momentum equations (the paper's equations have none; the
f-plane workloads need them).

The pressure follows from the ideal gas and the Exner definition,
p = p00 (R_d rho theta / p00)^(c_p/c_v), and the reference pressure is the same
function of the reference density and potential temperature, so that the
perturbation is p' = p(rho, theta) - p(rho0, theta0).  The oracle evaluates
that difference in x87 extended precision (64-bit significand) and rounds the
result to FP64, which removes the cancellation of two ~1e5 Pa numbers.

Discretisation (Section 3): collocation at the LGL nodes of each element,
1-D derivatives by the LGL derivative matrix along each tensor direction,
affine box elements with metric 2/dx, 2/dy, 2/dz.
"""

import numpy as np

from .gll import derivative_matrix

FIELDS = ("rho_p", "u", "v", "w", "theta_p")


def pressure_perturbation(rho0, theta0, rho_p, theta_p, R_d, c_p, p00):
    """p' = p00 (R_d rho theta/p00)^gamma - p00 (R_d rho0 theta0/p00)^gamma."""
    ld = np.longdouble
    Rd, cp, P0 = ld(R_d), ld(c_p), ld(p00)
    gamma = cp / (cp - Rd)
    rho = ld(1.0) * np.asarray(rho0, dtype=ld) + np.asarray(rho_p, dtype=ld)
    th = np.asarray(theta0, dtype=ld) + np.asarray(theta_p, dtype=ld)
    p = P0 * (Rd * rho * th / P0) ** gamma
    pref = P0 * (Rd * np.asarray(rho0, dtype=ld) * np.asarray(theta0, dtype=ld) / P0) ** gamma
    return (p - pref).astype(np.float64)


def local_derivatives(D, f, dx, dy, dz):
    """Tensor-product derivatives of element-local fields of shape (E,k,j,i).

    d/dx at (i,j,k) = (2/dx_e) sum_m D[i,m] f[m,j,k], likewise y (index j)
    and z (index k)."""
    two = f.dtype.type(2.0)
    fx = np.einsum("im,ekjm->ekji", D, f) * (two / dx)[:, None, None, None]
    fy = np.einsum("jm,ekmi->ekji", D, f) * (two / dy)[:, None, None, None]
    fz = np.einsum("km,emji->ekji", D, f) * (two / dz)[:, None, None, None]
    return fx, fy, fz


def element_rhs(mesh, qL, rho0, theta0, dtheta0dz, phys, dtype=np.float64):
    """Pointwise strong-form right-hand side on every local node.

    qL : array (5, E, n, n, n) of local values (rho', u, v, w, theta').
    rho0, theta0, dtheta0dz : reference state at the local nodes, (E,n,n,n).
    phys : dict with f, g, R_d, c_p, p00.
    dtype : float64, or float32 for the reduced-precision variant: the
            pointwise fields, the derivatives and the right-hand side are
            float32 arrays (perturbations and reference rounded to float32;
            p' is the exact difference rounded to float32, so no cancellation
            enters); the caller's assembly stays FP64.
    Returns R_L of shape (5, E, n, n, n) (not mass weighted, float64)."""
    pp = pressure_perturbation(rho0, theta0, qL[0], qL[4],
                               phys["R_d"], phys["c_p"], phys["p00"]).astype(dtype)
    qL = np.asarray(qL).astype(dtype)
    rho0, theta0, dtheta0dz = (np.asarray(a).astype(dtype) for a in (rho0, theta0, dtheta0dz))
    rho_p, u, v, w, th_p = qL
    D = derivative_matrix(mesh.N).astype(dtype)
    dx, dy, dz = (np.asarray(a).astype(dtype) for a in (mesh.e_dx, mesh.e_dy, mesh.e_dz))
    rho = rho0 + rho_p
    d = lambda f: local_derivatives(D, f, dx, dy, dz)
    mx, _, _ = d(rho * u)
    _, my, _ = d(rho * v)
    _, _, mz = d(rho * w)
    ux, uy, uz = d(u)
    vx, vy, vz = d(v)
    wx, wy, wz = d(w)
    px, py, pz = d(pp)
    tx, ty, tz = d(th_p)
    f, g = dtype(phys["f"]), dtype(phys["g"])
    R = np.empty_like(qL)
    R[0] = -(mx + my + mz)
    R[1] = -(u * ux + v * uy + w * uz) - px / rho + f * v
    R[2] = -(u * vx + v * vy + w * vz) - py / rho - f * u
    R[3] = -(u * wx + v * wy + w * wz) - pz / rho - (rho_p / rho) * g
    R[4] = -(u * tx + v * ty + w * tz) - w * dtheta0dz
    R = R.astype(np.float64)
    if phys.get("Cs", 0.0) > 0.0 or phys.get("sponge_gamma", 0.0) > 0.0:
        R += dissipation(mesh, np.asarray(qL, dtype=np.float64), phys)
    return R


def sponge_profile(z, z_top, gamma, depth):
    """Rayleigh absorbing layer of the paper's model setup (Section 5):
    R(z) = min(1, max(0, gamma sin^2(pi/2 (1 - (z_top - z)/depth)))) inside the
    top layer z >= z_top - depth, zero below it (the printed formula is
    garbled; below the layer its sine would not vanish)."""
    z = np.asarray(z, dtype=np.float64)
    arg = 0.5 * np.pi * (1.0 - (z_top - z) / depth)
    r = np.minimum(1.0, np.maximum(0.0, gamma * np.sin(arg) ** 2))
    return np.where(z >= z_top - depth, r, 0.0)


def dissipation(mesh, qL, phys):
    """Sub-grid and absorbing-layer tendencies (Section 5 model setup), FP64.

    Smagorinsky-Lilly in the horizontal: the momentum equations gain the
    horizontal divergence of 2 nu_t S, S = (grad u + grad u^T)/2 from the
    element-local derivatives, nu_t = (C_s Delta)^2 sqrt(2 S:S) with Delta the
    mean horizontal node spacing of the element, (dx + dy) / (2N):
        R_u += d/dx(2 nu S_xx) + d/dy(2 nu S_xy)
        R_v += d/dx(2 nu S_yx) + d/dy(2 nu S_yy)
        R_w += d/dx(2 nu S_zx) + d/dy(2 nu S_zy)
    (strong form inside each element, like every other term).  Rayleigh
    layer: every perturbation field gains -R(z) q'.
    phys keys: Cs (0 disables), sponge_gamma [1/s] (0 disables),
    sponge_depth [m]; the layer sits under the domain top."""
    D = derivative_matrix(mesh.N)
    d = lambda f: local_derivatives(D, f, mesh.e_dx, mesh.e_dy, mesh.e_dz)
    out = np.zeros_like(qL)
    cs = phys.get("Cs", 0.0)
    if cs > 0.0:
        u, v, w = qL[1], qL[2], qL[3]
        ux, uy, uz = d(u)
        vx, vy, vz = d(v)
        wx, wy, wz = d(w)
        sxx, syy, szz = ux, vy, wz
        sxy, sxz, syz = 0.5 * (uy + vx), 0.5 * (uz + wx), 0.5 * (vz + wy)
        ss = sxx**2 + syy**2 + szz**2 + 2.0 * (sxy**2 + sxz**2 + syz**2)
        delta = (mesh.e_dx + mesh.e_dy) / (2.0 * mesh.N)
        nu = (cs * delta)[:, None, None, None] ** 2 * np.sqrt(2.0 * ss)
        txx, txy, tyy, txz, tyz = (2.0 * nu * a for a in (sxx, sxy, syy, sxz, syz))
        out[1] += d(txx)[0] + d(txy)[1]
        out[2] += d(txy)[0] + d(tyy)[1]
        out[3] += d(txz)[0] + d(tyz)[1]
    gam = phys.get("sponge_gamma", 0.0)
    if gam > 0.0:
        rz = sponge_profile(mesh.zl, mesh.z_edges[-1], gam, phys.get("sponge_depth", 4000.0))
        out -= rz[None] * qL
    return out
