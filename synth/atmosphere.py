"""Synthetic background atmosphere and vortex (inputs only).

Background: constant Brunt-Vaisala frequency N_bv over a surface potential
temperature theta_s, in hydrostatic balance:

    theta0(z) = theta_s exp(N^2 z / g)
    pi0(z)    = 1 + g^2 / (c_p theta_s N^2) (exp(-N^2 z / g) - 1)
    rho0(z)   = p00 pi0^(c_v/R_d) / (R_d theta0)
    dtheta0/dz= theta0 N^2 / g

Vortex: axisymmetric about the domain centre, tangential wind
v(r, z) = V(r) T(r) Zv(z) with a modified-Rankine V (linear to V_max at r_max,
then V_max (r_max/r)^0.5), the paper's sixth-power radial taper
T = exp(-(r/D2)^6) with D2 = L/4 (which makes the field periodic to e^-64),
and a linear vertical decay Zv = max(0, 1 - z/z_v).  The pressure perturbation
is in gradient-wind balance with the reference density,
dp'/dr = rho0(z) (v^2/r + f v), integrated inward from r = L/2 where p' = 0;
the density perturbation is hydrostatic, rho' = -(1/g) dp'/dz; theta' follows
from the ideal-gas state (rho0 + rho', p0 + p'), plus seeded uniform noise
applied at fixed pressure (the density compensates).
"""

import numpy as np

from . import noise


def background(z, theta_s, N_bv, g, R_d, c_p, p00):
    z = np.asarray(z, dtype=np.float64)
    c_v = c_p - R_d
    N2 = N_bv * N_bv
    theta0 = theta_s * np.exp(N2 * z / g)
    pi0 = 1.0 + g * g / (c_p * theta_s * N2) * (np.exp(-N2 * z / g) - 1.0)
    rho0 = p00 * pi0 ** (c_v / R_d) / (R_d * theta0)
    dtheta0 = theta0 * N2 / g
    # d rho0/dz = rho0 ((c_v/R_d) pi0'/pi0 - theta0'/theta0), pi0' = -g/(c_p theta0)
    dpi0 = -g / (c_p * theta0)
    drho0 = rho0 * ((c_v / R_d) * dpi0 / pi0 - dtheta0 / theta0)
    p0 = p00 * pi0 ** (c_p / R_d)
    return dict(theta0=theta0, pi0=pi0, rho0=rho0, dtheta0dz=dtheta0,
                drho0dz=drho0, p0=p0)


def rankine(r, v_max, r_max, tail=0.5):
    r = np.asarray(r, dtype=np.float64)
    inner = v_max * r / r_max
    outer = v_max * (r_max / np.maximum(r, 1e-30)) ** tail
    return np.where(r <= r_max, inner, outer)


def smooth_profile(r, v_max, r_max):
    """V = 2 V_max x / (1 + x^2), x = r / r_max: peak V_max at r_max, smooth
    vorticity 4 V_max / (r_max (1 + x^2)^2) (no jump at r_max)."""
    x = np.asarray(r, dtype=np.float64) / r_max
    return 2.0 * v_max * x / (1.0 + x * x)


class Vortex:
    """Tabulated radial integrals of the balanced vortex."""

    def __init__(self, v_max, r_max, D2, R_out, z_top_v, f, n_tab=400001, profile="rankine"):
        self.v_max, self.r_max, self.D2 = v_max, r_max, D2
        self.profile = profile
        self.R_out, self.z_top_v, self.f = R_out, z_top_v, f
        # radial grid with r_max on a grid point
        n1 = max(2, int(round((n_tab - 1) * r_max / R_out)))
        r1 = np.linspace(0.0, r_max, n1 + 1)
        r2 = np.linspace(r_max, R_out, n_tab - n1)[1:]
        self.r = np.concatenate([r1, r2])
        vt = self.vt_surface(self.r)
        s = np.maximum(self.r, 1e-30)
        fa = np.where(self.r > 0, vt * vt / s, 0.0)
        fb = vt
        dr = np.diff(self.r)
        # integrals from r to R_out (trapezoid, accumulated inward)
        ca = np.concatenate([[0.0], np.cumsum(0.5 * dr * (fa[1:] + fa[:-1]))])
        cb = np.concatenate([[0.0], np.cumsum(0.5 * dr * (fb[1:] + fb[:-1]))])
        self.A = ca[-1] - ca
        self.B = cb[-1] - cb

    def vt_surface(self, r):
        prof = smooth_profile if self.profile == "smooth" else rankine
        return prof(r, self.v_max, self.r_max) * np.exp(-(np.asarray(r) / self.D2) ** 6)

    def zv(self, z):
        return np.maximum(0.0, 1.0 - np.asarray(z) / self.z_top_v)

    def dzv(self, z):
        return np.where(np.asarray(z) < self.z_top_v, -1.0 / self.z_top_v, 0.0)

    def integrals(self, r):
        r = np.asarray(r)
        A = np.interp(r, self.r, self.A, right=0.0)
        B = np.interp(r, self.r, self.B, right=0.0)
        return A, B

    def vorticity_surface(self, r, h=1.0):
        """zeta = (1/r) d(r v)/dr at z = 0 (central difference)."""
        r = np.maximum(np.asarray(r, dtype=np.float64), 2 * h)
        rv = lambda s: s * self.vt_surface(s)
        return (rv(r + h) - rv(r - h)) / (2 * h) / r


def smooth_modes(xyz, Lx, Ly, seed, n_modes=6, k_max=4):
    """A smooth periodic field in [-1, 1]: a normalised sum of n_modes
    horizontal Fourier modes (wavenumbers 1..k_max per direction) with seeded
    amplitudes and phases (PCG64), each with a seeded vertical half-sine."""
    rng = np.random.default_rng(seed)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    H = max(float(np.max(z)), 1.0)
    out = np.zeros_like(x)
    tot = 0.0
    for _ in range(n_modes):
        kx, ky = rng.integers(1, k_max + 1, size=2)
        ph = rng.uniform(0, 2 * np.pi, size=2)
        a = rng.uniform(0.5, 1.0)
        m = rng.integers(1, 3)
        out += a * np.cos(2 * np.pi * kx * x / Lx + ph[0]) * np.cos(2 * np.pi * ky * y / Ly + ph[1]) \
            * np.sin(m * np.pi * z / H)
        tot += a
    return out / tot


def initial_state(xyz, bg_fn, vortex, phys, noise_amp, noise_ztop, seed, Lx, Ly,
                  center=(0.0, 0.0), noise_kind="nodes"):
    """(rho', u, v, w, theta') at points xyz (n, 3)."""
    x, y, z = xyz[:, 0] - center[0], xyz[:, 1] - center[1], xyz[:, 2]
    g, R_d, c_p, p00 = phys["g"], phys["R_d"], phys["c_p"], phys["p00"]
    c_v = c_p - R_d
    bg = bg_fn(z)
    r = np.sqrt(x * x + y * y)
    Zv, dZv = vortex.zv(z), vortex.dzv(z)
    vt = vortex.vt_surface(r) * Zv
    rs = np.where(r > 0, r, 1.0)
    u = np.where(r > 0, -vt * y / rs, 0.0)
    v = np.where(r > 0, vt * x / rs, 0.0)
    A, B = vortex.integrals(r)
    f = vortex.f
    S = Zv * Zv * A + f * Zv * B
    dS = 2.0 * Zv * dZv * A + f * dZv * B
    p_p = -bg["rho0"] * S
    dp_dz = -bg["drho0dz"] * S - bg["rho0"] * dS
    rho_p = -dp_dz / g
    rho = bg["rho0"] + rho_p
    p = bg["p0"] + p_p
    theta = p00 / (R_d * rho) * (p / p00) ** (c_v / c_p)
    theta_p = theta - bg["theta0"]
    if noise_amp > 0.0:
        # perturb theta at fixed pressure: rho theta stays fixed, so the noise
        # is a buoyancy perturbation and not a pressure (acoustic) one
        if noise_kind == "modes":
            dth = noise_amp * smooth_modes(xyz, Lx, Ly, seed)
        else:
            U = noise.uniform01(xyz, Lx, Ly, seed)
            mask = z <= noise_ztop + 1e-6
            dth = np.where(mask, noise_amp * (2.0 * U - 1.0), 0.0)
        rho_new = rho * theta / (theta + dth)
        rho_p = rho_new - bg["rho0"]
        theta_p = theta_p + dth
    w = np.zeros_like(u)
    return np.stack([rho_p, u, v, w, theta_p])
