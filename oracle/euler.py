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
    return R.astype(np.float64)
