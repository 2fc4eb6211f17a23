"""Pins of the oracle's terrain-following (mapped) elements.

* flat terrain reduces to the box-element right-hand side of Section 3;
* the chain rule differentiates fields linear in the physical coordinates
  exactly, whatever the terrain (a wrong sign or index in the metric breaks it);
* the mapped lumped masses integrate the domain under the terrain exactly for
  a polynomial surface (LGL quadrature is exact at that degree);
* a manufactured solution over smooth terrain converges spectrally in N;
* on a plane slope the surface normal is exact and the bottom tendency is
  tangent to the surface.
"""

import numpy as np
import pytest

from oracle import assembly, terrain
from oracle.mesh import OracleMesh
from synth import cases, columns

from test_oracle_rhs import exact_rhs, manufactured


def build(c):
    return OracleMesh(c["N"], c["nx0"], c["ny0"], c["Lx"], c["Ly"], c["z_edges"],
                      c["columns"], c["periodic_x"], c["periodic_y"])


def ref_global(c, m, zsG):
    bg = cases.reference_state(c, terrain.node_heights(m, zsG))
    return dict(rho0=bg["rho0"], theta0=bg["theta0"], dtheta0dz=bg["dtheta0dz"])


def hills(c, amp=1500.0):
    """Smooth hills periodic over the domain in x and in y."""
    kx, ky = 2 * np.pi / c["Lx"], 2 * np.pi / c["Ly"]
    return lambda x, y: 0.5 * amp * (1.0 + np.cos(kx * x) * np.cos(ky * y + 0.4))


def test_flat_terrain_is_the_box_element_rhs():
    c = cases.get("vortex_8x8x4_n4")
    m = build(c)
    q = cases.initial_state(c, m.node_xyz)
    zs = np.zeros(m.n_dof)
    bg = cases.reference_state(c, m.zl)
    want = assembly.rhs(m, q, dict(rho0=bg["rho0"], theta0=bg["theta0"],
                                   dtheta0dz=bg["dtheta0dz"]), c["phys"])
    got = terrain.rhs(m, q, ref_global(c, m, zs), zs, c["phys"])
    scale = np.abs(want).max(axis=1, keepdims=True)
    assert np.all(np.abs(got - want) <= 1e-12 * scale)


@pytest.mark.parametrize("N", [2, 4, 7])
def test_linear_fields_differentiate_exactly(N):
    c = cases.get("vortex_8x8x4_n4", N=N)
    m = build(c)
    zs = hills(c)(m.node_xyz[:, 0], m.node_xyz[:, 1])
    zp = terrain.physical_z(m, zs)
    _, Jinv, detJ = terrain.jacobian(m, zp)
    assert np.all(detJ > 0)
    a, b, cz = 3e-4, -7e-4, 2e-3
    f = a * m.xl + b * m.yl + cz * zp
    gx, gy, gz = terrain.gradient(m, Jinv, f)
    for got, want in ((gx, a), (gy, b), (gz, cz)):
        assert np.abs(got - want).max() <= 1e-11 * abs(cz)
    # the height itself: grad z = (0, 0, 1) although z varies along x and y
    zx, zy, zz = terrain.gradient(m, Jinv, zp)
    assert np.abs(zx).max() < 1e-12 and np.abs(zy).max() < 1e-12
    assert np.abs(zz - 1.0).max() < 1e-12


@pytest.mark.parametrize("N", [2, 4])
def test_mapped_masses_integrate_the_volume_under_polynomial_terrain(N):
    c = cases.get("small_uniform", N=N)
    c["periodic_x"] = c["periodic_y"] = False
    m = build(c)
    Lx, Ly = c["Lx"], c["Ly"]
    A, B, C, Dxy, E = 900.0, 2e-3, -1e-3, 3e-8, 4e-8
    zs_fn = lambda x, y: A + B * x + C * y + Dxy * x * y + E * x * x
    zs = zs_fn(m.node_xyz[:, 0], m.node_xyz[:, 1])
    _, _, detJ = terrain.jacobian(m, terrain.physical_z(m, zs))
    mL, MG = terrain.lumped_mass(m, detJ)
    H = c["z_edges"][-1] - c["z_edges"][0]
    exact = H * Lx * Ly - (A * Lx * Ly + E * Lx**3 * Ly / 12.0)
    assert abs(mL.sum() - exact) <= 1e-12 * exact
    assert abs(MG.sum() - exact) <= 1e-12 * exact
    assert np.all(MG > 0)


def mms_error(N, nx, nz):
    L, H = 100e3, 10e3
    c = cases.get("vortex_8x8x4_n4")
    c.update(N=N, nx0=nx, ny0=nx, Lx=L, Ly=L, z_edges=np.linspace(0, H, nz + 1),
             columns=columns.uniform(nx, nx))
    m = build(c)
    zs = hills(c, amp=1200.0)(m.node_xyz[:, 0], m.node_xyz[:, 1])
    F = manufactured(L, H)
    xyz = m.node_xyz.copy()
    xyz[:, 2] = terrain.node_heights(m, zs)
    q = np.stack([Fi.val(*xyz.T) for Fi in F])
    R = terrain.rhs(m, q, ref_global(c, m, zs), zs, c["phys"])
    Rex = exact_rhs(c, xyz, F)
    inner = ~(terrain.surface_nodes(m) | terrain.top_nodes(m))
    scale = np.abs(Rex[:, inner]).max(axis=1)
    return (np.abs(R[:, inner] - Rex[:, inner]).max(axis=1) / scale).max()


def test_manufactured_solution_over_terrain_converges_spectrally():
    e = [mms_error(N, 4, 2) for N in (2, 4, 6, 8)]
    assert all(e[i + 1] < 0.2 * e[i] for i in range(3)), e
    assert e[-1] < 1e-4 * e[0], e


def test_plane_slope_normal_and_tangent_bottom_tendency():
    c = cases.get("vortex_8x8x4_n4")
    c["periodic_x"] = c["periodic_y"] = False
    m = build(c)
    s = 0.004
    zs = s * (m.node_xyz[:, 0] + 0.5 * c["Lx"])
    zp = terrain.physical_z(m, zs)
    _, Jinv, detJ = terrain.jacobian(m, zp)
    mL, MG = terrain.lumped_mass(m, detJ)
    n, bot = terrain.surface_normal(m, zs, Jinv, mL, MG)
    want = np.array([-s, 0.0, 1.0]) / np.sqrt(1 + s * s)
    assert np.abs(n - want[:, None]).max() < 1e-13
    xyz = m.node_xyz.copy()
    xyz[:, 2] = terrain.node_heights(m, zs)
    q = cases.initial_state(c, xyz)
    R = terrain.rhs(m, q, ref_global(c, m, zs), zs, c["phys"])
    normal = np.sum(R[1:4, bot] * n, axis=0)
    assert np.abs(normal).max() <= 1e-13 * np.abs(R[1:4, bot]).max()
    assert np.abs(R[1:4, bot]).max() > 0
    assert np.all(R[3, terrain.top_nodes(m)] == 0.0)


# ---------------------------------------------------------------- 2:1 meshes
def test_flat_terrain_is_the_box_element_rhs_on_nonconforming_meshes():
    for name, kw in (("small_amr2", {}), ("small_amr3", {"N": 5, "periodic": False})):
        c = cases.get(name, **kw)
        m = build(c)
        q = cases.initial_state(c, m.node_xyz)
        zs = np.zeros(m.n_dof)
        bg = cases.reference_state(c, m.zl)
        want = assembly.rhs(m, q, dict(rho0=bg["rho0"], theta0=bg["theta0"],
                                       dtheta0dz=bg["dtheta0dz"]), c["phys"])
        got = terrain.rhs(m, q, ref_global(c, m, zs), zs, c["phys"])
        scale = np.abs(want).max(axis=1, keepdims=True)
        assert np.all(np.abs(got - want) <= 1e-12 * scale), name


def test_nonconforming_geometry_is_watertight_and_exact_for_linear_fields():
    c = cases.get("small_amr3", N=4)
    m = build(c)
    zs = hills(c)(m.node_xyz[:, 0], m.node_xyz[:, 1])
    zp = terrain.physical_z(m, zs)
    # every local copy of a node (hanging copies included) has the height of
    # the coarse face's interpolant there: the mesh has no gaps
    zG = terrain.node_heights(m, zs)
    assert np.abs(zp.reshape(-1) - m.Z @ zG).max() < 1e-9
    _, Jinv, detJ = terrain.jacobian(m, zp)
    assert np.all(detJ > 0)
    a, b, cz = 3e-4, -7e-4, 2e-3
    gx, gy, gz = terrain.gradient(m, Jinv, a * m.xl + b * m.yl + cz * zp)
    for got, want in ((gx, a), (gy, b), (gz, cz)):
        assert np.abs(got - want).max() <= 1e-11 * abs(cz)


def test_mapped_masses_on_nonconforming_mesh_integrate_polynomial_terrain():
    c = cases.get("small_amr3", N=3, periodic=False)
    m = build(c)
    Lx, Ly = c["Lx"], c["Ly"]
    A, E = 900.0, 4e-8
    zs = A + E * m.node_xyz[:, 0] ** 2
    _, _, detJ = terrain.jacobian(m, terrain.physical_z(m, zs))
    mL, MG = terrain.lumped_mass(m, detJ)
    H = c["z_edges"][-1] - c["z_edges"][0]
    exact = H * Lx * Ly - (A * Lx * Ly + E * Lx**3 * Ly / 12.0)
    assert abs(mL.sum() - exact) <= 1e-12 * exact
    assert abs(MG.sum() - exact) <= 1e-12 * exact


def test_balanced_state_over_hills_converges_spectrally():
    """A constant-N hydrostatic atmosphere at rest, written as perturbations
    about an isothermal reference, over hills: steady in the continuum.
    Discretely the residual (the vertical tendency and the horizontal
    pressure-gradient error that terrain-following coordinates are known
    for) is truncation error and decays spectrally with N; at N = 2 it is
    far from zero, so the pin is not trivially satisfied."""
    from synth import atmosphere
    res_w, res_h = [], []
    for N in range(2, 9):
        c = cases.get("small_uniform", N=N)
        c["periodic_x"] = c["periodic_y"] = True
        m = build(c)
        zs = hills(c, amp=1200.0)(m.node_xyz[:, 0], m.node_xyz[:, 1])
        zp = terrain.node_heights(m, zs)
        p = c["phys"]
        Rd, cp, g, p00 = p["R_d"], p["c_p"], p["g"], p["p00"]
        T0 = 250.0

        def iso(z):
            pr = p00 * np.exp(-g * z / (Rd * T0))
            th = T0 * (p00 / pr) ** (Rd / cp)
            return dict(rho0=pr / (Rd * T0), theta0=th, dtheta0dz=th * g / (cp * T0))
        ref = iso(zp)
        b = c["background"]
        st = atmosphere.background(zp, b["theta_s"], b["N_bv"], g, Rd, cp, p00)
        q = np.zeros((5, m.n_dof))
        q[0] = st["rho0"] - ref["rho0"]
        q[4] = st["theta0"] - ref["theta0"]
        R = terrain.rhs(m, q, ref, zs, p)
        inner = ~(terrain.surface_nodes(m) | terrain.top_nodes(m))
        res_w.append(np.abs(R[3, inner]).max())
        res_h.append(np.abs(R[1:3, inner]).max())
    res_w, res_h = np.array(res_w), np.array(res_h)
    assert res_w[0] > 1e-4 and res_h[0] > 1e-5          # not balanced discretely at N = 2
    assert res_w[-1] < 1e-5 * res_w[0]
    assert res_h[-1] < 1e-3 * res_h[0]                   # pressure-gradient error: 3e-3 -> 4e-7
    assert np.all(np.diff(np.log(res_h)) < 0)           # decays at every order


def test_terrain_vorticity_of_solid_body_rotation_and_sheared_wind():
    """u = -W y, v = W x has vorticity 2W everywhere, over any terrain; and a
    wind v = a z (linear in the physical height) has none, although in the
    terrain-following coordinates v varies along x over a slope."""
    c = cases.get("small_amr3", N=4, periodic=False)
    m = build(c)
    W = 3e-4
    q = np.zeros((5, m.n_dof))
    q[1] = -W * m.node_xyz[:, 1]
    q[2] = W * m.node_xyz[:, 0]
    zs = hills(c)(m.node_xyz[:, 0], m.node_xyz[:, 1])
    zeta = terrain.criterion_vorticity(m, assembly.scatter(m, q), zs)
    assert np.abs(zeta - 2 * W).max() < 1e-9 * W
    zs = 0.004 * (m.node_xyz[:, 0] + 0.5 * c["Lx"])
    q = np.zeros((5, m.n_dof))
    q[2] = 1e-3 * terrain.node_heights(m, zs)
    zeta = terrain.criterion_vorticity(m, assembly.scatter(m, q), zs)
    assert np.abs(zeta).max() < 1e-12


@pytest.mark.parametrize("name", ["vortex_8x8x4_n4", "small_amr2"])
def test_fp32_mode_is_float32_arithmetic_over_terrain(name):
    """The mapped elements' reduced-precision mode really rounds to float32:
    over hills its tendency differs from FP64 by float32 round-off amplified by
    the derivatives (between 1e-9 and 1e-3 relative per field), on a uniform
    and a 2:1 mesh; a state at rest keeps a zero tendency in both modes (every
    term is a product with a vanishing perturbation or its derivative)."""
    from oracle import metrics
    c = cases.get(name)
    m = build(c)
    zs = hills(c)(m.node_xyz[:, 0], m.node_xyz[:, 1])
    ref = ref_global(c, m, zs)
    xyz = m.node_xyz.copy()
    xyz[:, 2] = terrain.node_heights(m, zs)
    q = cases.initial_state(c, xyz)
    r64 = terrain.rhs(m, q, ref, zs, c["phys"])
    r32 = terrain.rhs(m, q, ref, zs, c["phys"], dtype=np.float32)
    err = metrics.rel_l2(r32, r64, metrics.RHS_FLOORS)
    assert np.all(err > 1e-9) and np.all(err < 1e-3), err
    rest = np.zeros_like(q)
    for dt in (np.float64, np.float32):
        assert np.abs(terrain.rhs(m, rest, ref, zs, c["phys"], dtype=dt)).max() == 0.0


def test_flat_terrain_features_are_the_box_features():
    """The forecaster features over flat terrain reduce to the box-element
    ones (the chain rule with the identity mapping)."""
    from oracle import forecast
    c = cases.get("small_amr2")
    m = build(c)
    q = cases.initial_state(c, m.node_xyz)
    rng = np.random.default_rng(3)
    qp = q * (1.0 + 0.05 * rng.standard_normal(q.shape))
    qL, qLp = assembly.scatter(m, q), assembly.scatter(m, qp)
    bg = cases.reference_state(c, m.zl)
    refL = dict(rho0=bg["rho0"], theta0=bg["theta0"])
    plain = rng.integers(-1, 2, size=m.n_elem)
    thr, scale = [1e-4, 3e-4], np.ones(16)
    box, dbox = forecast.features(m, qL, qLp, plain, refL, c["phys"], 1, thr, 2, scale)
    ter, dter = forecast.features(m, qL, qLp, plain, refL, c["phys"], 1, thr, 2, scale,
                                  zsG=np.zeros(m.n_dof))
    assert np.all(np.abs(ter - box) <= 1e-12 * (np.abs(box).max(0) + 1e-300))
    np.testing.assert_array_equal(dter, dbox)


@pytest.mark.parametrize("name", ["vortex_8x8x4_n4", "small_amr2"])
def test_terrain_features_of_linear_fields_are_exact(name):
    """Winds and theta' linear in the physical coordinates over hills:
    max|zeta| = mean zeta = 2 Omega, max|div u| = |a + b + c| and
    max|grad theta'| = |(g1, g2, g3)| in every element, whatever the terrain
    (a wrong metric term, sign or index in the chain rule breaks them)."""
    from oracle import forecast
    c = cases.get(name)
    m = build(c)
    zs = hills(c)(m.node_xyz[:, 0], m.node_xyz[:, 1])
    zp = terrain.physical_z(m, zs)
    om_, a, b, cz = 2e-4, 3e-5, -5e-5, 1e-4
    g1, g2, g3 = 2e-6, -1e-6, 4e-3
    x, y = m.xl, m.yl
    qL = np.stack([np.zeros_like(x), a * x - om_ * y, om_ * x + b * y, cz * zp,
                   g1 * x + g2 * y + g3 * zp])
    bg = cases.reference_state(c, zp.reshape(-1))
    refL = dict(rho0=bg["rho0"].reshape(x.shape), theta0=bg["theta0"].reshape(x.shape))
    F, _ = forecast.features(m, qL, qL, np.zeros(m.n_elem), refL, c["phys"], 1, [1.0, 2.0], 2,
                             np.ones(16), zsG=zs)
    np.testing.assert_allclose(F[:, 1], 2 * om_, rtol=1e-10)
    np.testing.assert_allclose(F[:, 2], 2 * om_, rtol=1e-10)
    np.testing.assert_allclose(F[:, 9], abs(a + b + cz), rtol=1e-9)
    np.testing.assert_allclose(F[:, 8], np.sqrt(g1 ** 2 + g2 ** 2 + g3 ** 2), rtol=1e-10)
    # the box derivatives would see the terrain's slope in theta' and w
    Fb, _ = forecast.features(m, qL, qL, np.zeros(m.n_elem), refL, c["phys"], 1, [1.0, 2.0], 2,
                              np.ones(16))
    assert np.abs(Fb[:, 8] - F[:, 8]).max() > 1e-3 * F[:, 8].max()


def _diss_phys(c, cs=0.21, gamma=0.01, depth=4000.0):
    ph = dict(c["phys"])
    ph.update(Cs=cs, sponge_gamma=gamma, sponge_depth=depth)
    return ph


def test_flat_terrain_with_dissipation_is_the_box_element_rhs():
    """Flat terrain with the Smagorinsky and absorbing-layer terms reduces to
    the box-element right-hand side with the same terms (uniform and 2:1)."""
    for name in ("vortex_8x8x4_n4", "small_amr2"):
        c = cases.get(name)
        m = build(c)
        q = cases.initial_state(c, m.node_xyz)
        ph = _diss_phys(c)
        zs = np.zeros(m.n_dof)
        bg = cases.reference_state(c, m.zl)
        want = assembly.rhs(m, q, dict(rho0=bg["rho0"], theta0=bg["theta0"],
                                       dtheta0dz=bg["dtheta0dz"]), ph)
        got = terrain.rhs(m, q, ref_global(c, m, zs), zs, ph)
        scale = np.abs(want).max(axis=1, keepdims=True)
        assert np.all(np.abs(got - want) <= 1e-12 * scale)
        # the terms are really on: without them the result differs
        plain = terrain.rhs(m, q, ref_global(c, m, zs), zs, c["phys"])
        assert np.abs(plain - got).max(axis=1)[1:4].min() > 1e-6 * scale[1:4].min()


@pytest.mark.parametrize("name", ["vortex_8x8x4_n4", "small_amr2"])
def test_uniform_strain_over_terrain_has_no_subgrid_tendency(name):
    """Winds linear in the physical coordinates have a uniform strain rate,
    hence a uniform stress with zero divergence: the sub-grid tendency
    vanishes over hills (box derivatives would see a non-uniform strain)."""
    c = cases.get(name)
    m = build(c)
    zs = hills(c)(m.node_xyz[:, 0], m.node_xyz[:, 1])
    zp = terrain.physical_z(m, zs)
    _, Jinv, _ = terrain.jacobian(m, zp)
    x, y = m.xl, m.yl
    qL = np.stack([np.zeros_like(x), 3e-5 * x - 2e-4 * y + 1e-3 * zp, 2e-4 * x + 5e-5 * y,
                   -8e-5 * zp + 1e-6 * x, np.zeros_like(x)])
    ph = _diss_phys(c, gamma=0.0)
    out = terrain.dissipation(m, qL, ph, Jinv, zp)
    # scale: the stress divided by the element width
    delta = (m.e_dx + m.e_dy).max() / (2.0 * m.N)
    tau = 2.0 * (0.21 * delta) ** 2 * 1e-3 * 1e-3
    assert np.abs(out).max() <= 1e-9 * tau / m.e_dz.min()
    from oracle.euler import dissipation as box_dissipation
    assert np.abs(box_dissipation(m, qL, ph)[1:4]).max() > 1e-3 * tau / m.e_dz.min()


def test_absorbing_layer_follows_the_physical_height():
    """The layer coefficient at the domain top is min(1, gamma) in every
    column (there the mapping leaves the height unchanged), and it reaches
    nodes whose flat height is below the layer when the terrain lifts them
    into it."""
    c = cases.get("vortex_8x8x4_n4")
    m = build(c)
    H, depth, gamma = m.z_edges[-1], 7000.0, 0.02
    zs = hills(c, amp=3000.0)(m.node_xyz[:, 0], m.node_xyz[:, 1])
    zp = terrain.physical_z(m, zs)
    _, Jinv, _ = terrain.jacobian(m, zp)
    qL = np.ones((5,) + m.local_shape())
    out = terrain.dissipation(m, qL, _diss_phys(c, cs=0.0, gamma=gamma, depth=depth), Jinv, zp)
    rz = -out[0]
    top = np.abs(m.zl - H) < 1e-9 * H
    np.testing.assert_allclose(rz[top], min(1.0, gamma), rtol=1e-12)
    assert np.all(rz[zp < H - depth] == 0.0)
    lifted = (m.zl < H - depth) & (zp > H - depth + 1.0)
    assert lifted.any() and np.all(rz[lifted] > 0.0)
    for f in range(5):
        assert np.array_equal(out[f], out[0])
