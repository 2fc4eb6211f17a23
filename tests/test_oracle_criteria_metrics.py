"""Pins of the refinement criteria (Section 4.1) and of the comparison
metrics (floor-scaled relative L2; maximum wind of Section 5.2).

Every expected value is a closed form or a number worked out by hand, never
a re-typing of the oracle's formula:

* criterion_vorticity: a solid-body rotation u = -W y, v = W x has vertical
  vorticity dv/dx - du/dy = 2 W at every point; a shear u = S y has -S; a
  pure strain u = a x, v = -a y has 0.  The fields are linear, so the LGL
  derivatives are exact on every element, including the fine elements of a
  2:1 mesh.
* criterion_speed: |(u, v, w)| of a constant field (3, 4, 12) is 13, and of
  u = x (v = w = 0) it is |x|.
* rel_l2: hand-computed two-field cases, one where the floor s_f sqrt(n)
  decides the denominator and one where ||b|| does.
* max_wind: nodes inside, on and outside the edge of the box.
"""

import numpy as np
import pytest

from oracle import amr, metrics
from oracle.mesh import OracleMesh
from synth import cases


def _mesh(name, **kw):
    c = cases.get(name, **kw)
    return OracleMesh(c["N"], c["nx0"], c["ny0"], c["Lx"], c["Ly"], c["z_edges"], c["columns"],
                      c["periodic_x"], c["periodic_y"])


def _local_state(m, u, v, w=None):
    q = np.zeros((5,) + m.xl.shape)
    q[1], q[2] = u, v
    if w is not None:
        q[3] = w
    return q


# the 2:1 meshes have fine columns around the centre; their elements are
# half as wide, which a wrong metric factor would expose
MESHES = [("vortex_8x8x4_n4", {}), ("small_amr2", {}), ("small_amr3", {"N": 5})]


@pytest.mark.parametrize("name,kw", MESHES)
@pytest.mark.parametrize("W", [1e-4, -3e-3])
def test_vorticity_of_solid_body_rotation(name, kw, W):
    m = _mesh(name, **kw)
    assert m.max_level >= (0 if name.startswith("vortex") else 1)
    C = amr.criterion_vorticity(m, _local_state(m, -W * m.yl, W * m.xl))
    np.testing.assert_allclose(C, 2.0 * W, rtol=1e-9, atol=0)


@pytest.mark.parametrize("name,kw", MESHES)
def test_vorticity_of_shear_and_strain(name, kw):
    m = _mesh(name, **kw)
    S = 2.5e-4
    C = amr.criterion_vorticity(m, _local_state(m, S * m.yl, np.zeros_like(m.xl)))
    np.testing.assert_allclose(C, -S, rtol=1e-9, atol=0)
    a = 7e-4
    C = amr.criterion_vorticity(m, _local_state(m, a * m.xl, -a * m.yl))
    # |dv/dx| and |du/dy| are zero exactly up to rounding of the node sums
    assert np.abs(C).max() < 1e-12 * a * 1e3


@pytest.mark.parametrize("name,kw", MESHES[:2])
def test_speed_of_constant_and_linear_fields(name, kw):
    m = _mesh(name, **kw)
    one = np.ones_like(m.xl)
    C = amr.criterion_speed(_local_state(m, 3.0 * one, 4.0 * one, 12.0 * one))
    np.testing.assert_allclose(C, 13.0, rtol=1e-15)
    C = amr.criterion_speed(_local_state(m, 1e-3 * m.xl, 0 * one, 0 * one))
    np.testing.assert_allclose(C, 1e-3 * np.abs(m.xl), rtol=1e-15, atol=0)
    # the vertical component counts: (0, 0, -2) has speed 2
    C = amr.criterion_speed(_local_state(m, 0 * one, 0 * one, -2.0 * one))
    np.testing.assert_allclose(C, 2.0, rtol=0)


def test_speed_criterion_drives_flags_like_the_text_rule():
    """|u| = 13 everywhere with thresholds (10, 20): a level-0 element refines
    (13 > 10), a level-1 element keeps (10 < 13 <= 20), a level-2 element at
    lvl_max = 2 coarsens only if 13 <= threshold(2) = 20, which holds."""
    C = np.full((3, 8), 13.0)
    out = amr.element_flags(C, np.array([0, 1, 2]), [10.0, 20.0], 2)
    assert out.tolist() == [1, 0, -1]


def test_rel_l2_floor_active():
    """b = 0: ||a - b|| = sqrt(3^2 + 4^2) = 5 and the denominator is the floor
    s sqrt(n) = 2 sqrt(2); second field: ||a - b|| = 1, floor 0.5 sqrt(2)."""
    a = np.array([[3.0, 4.0], [0.0, 1.0]])
    b = np.zeros((2, 2))
    out = metrics.rel_l2(a, b, np.array([2.0, 0.5]))
    assert out[0] == pytest.approx(5.0 / (2.0 * np.sqrt(2.0)), rel=1e-15)
    assert out[1] == pytest.approx(1.0 / (0.5 * np.sqrt(2.0)), rel=1e-15)


def test_rel_l2_floor_inactive_and_argument_order():
    """b = (6, 8): ||b|| = 10 exceeds the floor 1 sqrt(2), so the error of
    a = (3, 4) is 5 / 10; swapping the arguments gives 5 / 5."""
    a = np.array([[3.0, 4.0]])
    b = np.array([[6.0, 8.0]])
    assert metrics.rel_l2(a, b, np.array([1.0]))[0] == pytest.approx(0.5, rel=1e-15)
    assert metrics.rel_l2(b, a, np.array([1.0]))[0] == pytest.approx(1.0, rel=1e-15)
    # four nodes: the floor grows like sqrt(n): 1 * sqrt(4) = 2 > ||b|| = 1
    a4 = np.array([[1.0, 0.0, 0.0, 0.0]])
    b4 = np.array([[0.0, 1.0, 0.0, 0.0]])
    assert metrics.rel_l2(a4, b4, np.array([1.0]))[0] == pytest.approx(np.sqrt(2.0) / 2.0, rel=1e-15)


def test_max_wind_box_edges():
    """Nodes at |x|, |y| <= 50 km count, including the edge; a node 1 m
    outside does not, however fast."""
    xyz = np.array([[0.0, 0.0, 100.0],        # inside: (3, 4) -> 5
                    [50e3, -50e3, 0.0],       # on the corner: (6, 8) -> 10
                    [50001.0, 0.0, 0.0],      # outside in x: 100
                    [0.0, -50001.0, 5e3],     # outside in y: 200
                    [-20e3, 10e3, 1e3]])      # inside: (0, -7) -> 7
    q = np.zeros((5, 5))
    q[1] = [3.0, 6.0, 100.0, 0.0, 0.0]
    q[2] = [4.0, 8.0, 0.0, 200.0, -7.0]
    q[3] = [50.0, 50.0, 50.0, 50.0, 50.0]     # vertical wind is not part of it
    assert metrics.max_wind(xyz, q) == pytest.approx(10.0, rel=1e-15)
    assert metrics.max_wind(xyz, q, half_width=60e3) == pytest.approx(200.0, rel=1e-15)
    assert metrics.max_wind(xyz[[2, 3]], q[:, [2, 3]]) == 0.0
