"""Pins of the oracle mesh, hanging-node interpolation and DSS (Section 3.1)."""

import numpy as np
import pytest

from oracle.mesh import OracleMesh
from oracle import assembly
from synth import cases

MESHES = [("vortex_8x8x4_n4", {}), ("small_uniform", {"N": 3}), ("small_amr2", {}),
          ("small_amr2", {"N": 7}), ("small_amr3", {}), ("small_amr3", {"N": 7}),
          ("small_amr3", {"periodic": False}), ("small_amr3", {"periodic": False, "N": 7}),
          ("small_amr2", {"periodic": False, "N": 5})]


def build(name, kw):
    c = cases.get(name, **dict(kw))
    return c, OracleMesh(c["N"], c["nx0"], c["ny0"], c["Lx"], c["Ly"], c["z_edges"],
                         c["columns"], c["periodic_x"], c["periodic_y"])


@pytest.mark.parametrize("name,kw", MESHES)
def test_mass_sums_to_volume(name, kw):
    c, m = build(name, kw)
    per_elem = m.mL.reshape(m.n_elem, -1).sum(axis=1)
    np.testing.assert_allclose(per_elem, m.e_dx * m.e_dy * m.e_dz, rtol=1e-14)
    vol = c["Lx"] * c["Ly"] * (c["z_edges"][-1] - c["z_edges"][0])
    assert abs(m.MG.sum() / vol - 1) < 1e-13
    assert m.MG.min() > 0


@pytest.mark.parametrize("name,kw", MESHES)
def test_partition_of_unity_and_conservation(name, kw):
    """Rows of Z sum to one, so sum M_G R_G = sum m_L R_L for any local R."""
    c, m = build(name, kw)
    rs = np.asarray(m.Z.sum(axis=1)).ravel()
    np.testing.assert_allclose(rs, 1.0, atol=1e-13)
    rng = np.random.default_rng(3)
    RL = rng.standard_normal((2, m.n_loc))
    RG = assembly.gather(m, RL, lid_field=None)
    for f in range(2):
        a = np.dot(m.MG, RG[f])
        b = np.dot(m.mL, RL[f])
        assert abs(a - b) <= 1e-12 * np.dot(m.mL, np.abs(RL[f]))


def _poly(x, y, z, N, c):
    sx, sy, sz = x / c["Lx"], y / c["Ly"], z / c["z_edges"][-1]
    return (1.0 + sx - 0.7 * sx**N) * (0.5 - sy**N + 0.2 * sy**2) \
        + 0.3 * sx**(N - 1) * sy + sz**N * (1 + sx) - 2 * sz * sy**(N - 1)


@pytest.mark.parametrize("name,kw", [m for m in MESHES if m[1].get("periodic") is False])
def test_polynomial_reproduction_across_nc_faces(name, kw):
    """A global polynomial of degree <= N per direction, sampled at the unique
    nodes, is reproduced exactly at every hanging node by Z."""
    c, m = build(name, kw)
    N = m.N
    X, Y, Zc = m.node_xyz.T
    qG = _poly(X, Y, Zc, N, c)
    qL = m.Z @ qG
    ref = _poly(m.xl.ravel(), m.yl.ravel(), m.zl.ravel(), N, c)
    assert m.hanging.sum() > 0
    err = np.abs(qL - ref)[m.hanging].max()
    assert err < 1e-13 * np.abs(ref).max()
    # and a degree N+1 polynomial is NOT reproduced (the test can fail)
    hx, hy = c["Lx"] / c["nx0"], c["Ly"] / c["ny0"]
    qG2 = (X / hx) ** (N + 1) + (Y / hy) ** (N + 1)
    ref2 = (m.xl.ravel() / hx) ** (N + 1) + (m.yl.ravel() / hy) ** (N + 1)
    assert np.abs((m.Z @ qG2) - ref2)[m.hanging].max() > 1e-6


@pytest.mark.parametrize("name,kw", [MESHES[0], MESHES[1]])
def test_dss_identity_on_continuous_fields_conforming(name, kw):
    c, m = build(name, kw)
    rng = np.random.default_rng(1)
    r = rng.standard_normal((3, m.n_dof))
    back = assembly.gather(m, assembly.scatter(m, r).reshape(3, -1), lid_field=None)
    np.testing.assert_allclose(back, r, atol=1e-13)


@pytest.mark.parametrize("name,kw", MESHES[2:])
def test_dss_constants_on_nc(name, kw):
    c, m = build(name, kw)
    back = assembly.gather(m, assembly.scatter(m, np.full((1, m.n_dof), 2.5)).reshape(1, -1),
                           lid_field=None)
    np.testing.assert_allclose(back, 2.5, rtol=1e-13)


def test_unique_counts():
    """Counts fixed by the structure: (nx*N)(ny*N)(nz*N+1) periodic uniform."""
    c, m = build("vortex_8x8x4_n4", {})
    assert m.n_dof == 32 * 32 * 17 and m.hanging.sum() == 0
    c, m = build("small_uniform", {"N": 3})
    assert m.n_dof == (4 * 3) * (3 * 3) * (3 * 3 + 1)


def test_hanging_count_two_level_block():
    """6x6 base with a 2x3 block refined once (periodic, N=4): the block's
    boundary has 10 coarse edges, each carrying 2 fine edges with N-1
    hanging points, per vertical node (n_z N + 1 = 9 levels)."""
    c, m = build("small_amr2", {})
    assert m.n_hang_points == 10 * 2 * 3 * 9
    # odd N: the coarse-edge midpoint hangs as well (2(N-1)+1 per coarse edge)
    c, m = build("small_amr2", {"N": 7})
    assert m.n_hang_points == 10 * (2 * 6 + 1) * 15
