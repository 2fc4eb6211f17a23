"""Pins of the oracle forecaster's mesh side: features on fields whose
derivatives have closed forms, the neighbour sets of simple layouts, the
flag combination against a literal table, and hand-worked labels."""

import numpy as np

from harness import oracle_mesh
from oracle import assembly, forecast
from synth import cases


def setup(name, **kw):
    c = cases.get(name, **kw)
    m = oracle_mesh(c)
    ref = cases.reference_state(c, m.zl)
    return c, m, dict(rho0=ref["rho0"], theta0=ref["theta0"])


def test_solid_body_rotation_features():
    """u = -W y, v = W x (relative to the domain centre): zeta = 2W and
    div u = 0 at every node; theta' = a x + b z has |grad theta'| exact."""
    c, m, ref = setup("small_amr3", periodic=False)     # linear fields are not periodic
    X, Y, Z = m.node_xyz.T
    W, a, b = 1e-4, 2e-6, -3e-5
    q = np.zeros((5, m.n_dof))
    q[1], q[2] = -W * Y, W * X
    q[4] = a * X + b * Z
    qL = assembly.scatter(m, q)
    ones = np.ones(16)
    F, dem = forecast.features(m, qL, qL, np.zeros(m.n_elem), ref, c["phys"], 1, [1.5e-4], 1, ones)
    np.testing.assert_allclose(F[:, 1], 2 * W, rtol=1e-10)
    np.testing.assert_allclose(F[:, 2], 2 * W, rtol=1e-10)
    assert np.all(F[:, 9] < 1e-12 * W * 1e3)
    np.testing.assert_allclose(F[:, 8], np.hypot(a, b), rtol=1e-10)
    assert np.all(F[:, 13] == 0) and np.all(F[:, 14] == 0)
    np.testing.assert_array_equal(F[:, 0], m.e_level)
    assert np.all(dem == 1)              # 2W = 2e-4 > 1.5e-4
    # max|u_h| of an element is W times its farthest node from the centre
    r = np.hypot(m.xl, m.yl).reshape(m.n_elem, -1).max(1)
    np.testing.assert_allclose(F[:, 3], W * r, rtol=1e-12)


def test_scales_multiply_features():
    c, m, ref = setup("small_uniform", N=3)
    rng = np.random.default_rng(0)
    q = rng.standard_normal((5, m.n_dof)) * np.array([[1e-3], [1], [1], [0.1], [0.5]])
    qL = assembly.scatter(m, q)
    sc = rng.uniform(0.5, 2.0, 16)
    F1, _ = forecast.features(m, qL, qL * 0.9, np.ones(m.n_elem), ref, c["phys"], 0, [5.0], 1, np.ones(16))
    F2, _ = forecast.features(m, qL, qL * 0.9, np.ones(m.n_elem), ref, c["phys"], 0, [5.0], 1, sc)
    np.testing.assert_allclose(F2, F1 * sc[None, :], rtol=1e-15)


def test_neighbours_of_uniform_and_refined_layouts():
    c, m, _ = setup("vortex_8x8x4_n4")
    nb = forecast.neighbour_elements(m)
    assert all(len(x) == 8 for x in nb)          # periodic uniform: 8 around
    c, m, _ = setup("small_uniform", N=3)         # 4 x 3 periodic: wraps onto itself
    nb = forecast.neighbour_elements(m)
    assert all(len(x) == 8 for x in nb)
    # a refined column next to coarse ones: its 4 children see each other
    # and the coarse columns around, never elements of another layer
    c, m, _ = setup("small_amr2")
    nb = forecast.neighbour_elements(m)
    for e, x in enumerate(nb):
        assert all(m.e_layer[y] == m.e_layer[e] and m.e_col[y] != m.e_col[e] for y in x)
        assert len(x) >= 3


def test_flag_combination_table():
    rows = []
    for cls in range(3):
        for p in (-1, 0, 1):
            for lv in (0, 1, 2):
                rows.append((cls, p, lv))
    logits = np.zeros((len(rows), 3))
    for r, (cls, _, _) in enumerate(rows):
        logits[r, cls] = 1.0
    plain = np.array([p for _, p, _ in rows])
    lv = np.array([l for _, _, l in rows])
    # one column per element (n_z = 1); level-0 columns have no siblings
    cols = np.array([(0, r, 0) for r in range(len(rows))])
    e, _ = forecast.forecast_flags(logits, plain, lv, 2, cols, 1)
    for r, (cls, p, l) in enumerate(rows):
        f = cls - 1
        if f == 1 and l >= 2:
            f = 0
        if f == -1 and l == 0:
            f = 0
        want = 1 if (p == 1 or f == 1) else (-1 if (p == -1 and f == -1) else 0)
        assert e[r] == want, (cls, p, l)
    # ties go to the first maximum (coarsen before keep before refine)
    e, _ = forecast.forecast_flags(np.array([[1.0, 1.0, 0.0]]), [-1], [1], 2, [(1, 0, 0)], 1)
    assert e[0] == -1


def test_labels_hand_example():
    # 2 x 1 base, one layer; at t: (0,0,0) and the four children of (0,1,0)
    at = np.array([(0, 0, 0), (1, 2, 0), (1, 3, 0), (1, 2, 1), (1, 3, 1)])
    # later: (0,0,0) split, (0,1,0) merged back
    later = np.array([(1, 0, 0), (1, 1, 0), (1, 0, 1), (1, 1, 1), (0, 1, 0)])
    dem_later = np.array([2, 0, 1, 0, 0])
    lab = forecast.labels(at, later, dem_later, 1)
    # (0,0,0) covers four later columns, max dem 2 -> +1 (class 2); the
    # level-1 children sit inside (0,1,0) with dem 0 -> -1 (class 0)
    np.testing.assert_array_equal(lab, [2, 0, 0, 0, 0])
    lab = forecast.labels(at, later, np.array([0, 0, 0, 0, 1]), 1)
    np.testing.assert_array_equal(lab, [1, 1, 1, 1, 1])
