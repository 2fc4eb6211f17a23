"""Pins of the oracle's sub-grid (horizontal Smagorinsky-Lilly) and
absorbing-layer terms (the paper's model setup, Section 5):

* no strain, no sub-grid tendency (uniform wind: round-off only);
* a linear shear has constant strain, hence a constant stress and no
  tendency;
* a quadratic shear u = beta (y - y_s)^2 (y > y_s everywhere) has the closed
  form R_u = 8 (C_s Delta)^2 beta^2 (y - y_s) (every factor of nu_t and of the
  stress shows up in the 8), R_v = R_w = 0;
* the Rayleigh layer: the profile's closed form (zero below the layer, gamma
  capped at one at the top) and R = -R(z) q' for constant perturbations.
"""

import numpy as np

from harness import oracle_mesh
from oracle import assembly, euler
from synth import cases

PHYS = dict(cases.PHYS, f=0.0, Cs=0.21)


def mesh(N=4, periodic=False):
    c = cases.get("small_uniform", N=N)
    c["periodic_x"] = c["periodic_y"] = periodic
    return c, oracle_mesh(c)


def local(m, fields):
    return np.stack([m.Z @ f for f in fields]).reshape((len(fields),) + m.local_shape())


def test_no_strain_no_subgrid_tendency():
    c, m = mesh()
    q = np.zeros((5, m.n_dof))
    q[1], q[2] = 7.0, -3.0
    out = euler.dissipation(m, local(m, q), PHYS)
    assert np.abs(out).max() < 1e-25          # round-off of D applied to constants


def test_linear_shear_has_no_subgrid_tendency():
    c, m = mesh()
    X, Y, Z = m.node_xyz.T
    q = np.zeros((5, m.n_dof))
    q[1] = 2e-4 * Y
    q[2] = -1e-4 * X + 5e-5 * Y
    q[3] = 1e-6 * X
    out = euler.dissipation(m, local(m, q), PHYS)
    assert np.abs(out).max() < 1e-15


def test_quadratic_shear_closed_form():
    for N in (2, 4, 6):
        c, m = mesh(N)
        X, Y, Z = m.node_xyz.T
        beta, ys = 1e-9, -0.6 * c["Ly"]
        q = np.zeros((5, m.n_dof))
        q[1] = beta * (Y - ys) ** 2
        R = assembly.gather(m, euler.dissipation(m, local(m, q), PHYS), lid_field=None)
        delta = (m.e_dx[0] + m.e_dy[0]) / (2 * N)
        want = 8.0 * (0.21 * delta) ** 2 * beta**2 * (Y - ys)
        assert np.abs(R[1] - want).max() <= 1e-11 * np.abs(want).max()
        assert np.abs(R[[0, 2, 3, 4]]).max() <= 1e-13 * np.abs(want).max()


def test_sponge_profile_and_term():
    zt, depth = 20e3, 4e3
    z = np.array([0.0, 15.9e3, 16e3, 17e3, 18e3, 20e3])
    r = euler.sponge_profile(z, zt, 1.0, depth)
    np.testing.assert_allclose(r, [0, 0, 0, np.sin(np.pi / 8) ** 2, 0.5, 1.0], atol=1e-15)
    assert euler.sponge_profile(zt, zt, 3.0, depth) == 1.0        # capped at one
    c, m = mesh()
    q = np.zeros((5, m.n_dof)) + np.array([[1e-3], [2.0], [-1.0], [0.5], [0.3]])
    phys = dict(PHYS, Cs=0.0, sponge_gamma=0.7, sponge_depth=8e3)
    qL = local(m, q)
    out = euler.dissipation(m, qL, phys)
    rz = euler.sponge_profile(m.zl, m.z_edges[-1], 0.7, 8e3)
    np.testing.assert_allclose(out, -rz[None] * qL, rtol=0, atol=1e-16)
    assert np.abs(out).max() > 0
