"""Pins of the oracle's adaptation pass and solution transfer (Section 4.1,
with the readings for balance and transfer stated in ``oracle.adapt``).

What fixes them without an implementation to compare against:
* a hand-worked layout (a split that forces balance splits two cells away),
  a merge, and a merge blocked by a finer neighbour;
* structural invariants on random layouts and flags: cover without overlap,
  2:1 balance (brute force on the finest grid), every +1 column split,
  merges only of complete -1 families, and minimality of balance splits;
* transfer: identity on an unchanged layout, exact reproduction of a global
  polynomial of degree <= N on any adapted layout, the round trip
  split-then-merge returns any field exactly, and the lumped-mass integral
  is conserved by splits and by merges (interpolation of a degree-N
  polynomial and the mass-weighted projection are both exact for it).
"""

import numpy as np
import pytest

from oracle import adapt
from oracle.mesh import OracleMesh
from synth import columns as sc


def leafset(cols):
    if isinstance(cols, set):
        return set(cols)
    return {tuple(int(t) for t in c) for c in np.asarray(cols).reshape(-1, 3)}


def flags_for(cols, chosen):
    cols = [tuple(int(t) for t in c) for c in np.asarray(cols).reshape(-1, 3)]
    return np.array([chosen.get(c, 0) for c in cols], dtype=np.int8)


def covers(leaves, nx0, ny0):
    depth = max(l for l, _, _ in leaves)
    area = sum(4 ** (depth - l) for l, _, _ in leaves)
    m = adapt.finest_level_map(leaves, nx0, ny0, depth)
    return area == (nx0 << depth) * (ny0 << depth) and (m >= 0).all()


# ------------------------------------------------------------------ layouts
def test_no_flags_is_identity():
    for seed in range(4):
        cols = random_layout(seed, 4, 4, 3)
        out = adapt.adapt_columns(cols, np.zeros(len(cols), np.int8), 4, 4, 3)
        assert out == leafset(cols)


def test_split_forces_balance_two_cells_away():
    # 4x4 level-0 grid; (0,1,1) split earlier; now its child (1,3,3) (upper
    # right quarter) is split again: the level-0 cells east, north and
    # north-east of (0,1,1) touch level-2 leaves and must be split once.
    base = leafset(sc.uniform(4, 4)) - {(0, 1, 1)}
    base |= {(1, 2 + a, 2 + b) for a in (0, 1) for b in (0, 1)}
    cols = sorted(base)
    out = adapt.adapt_columns(cols, flags_for(cols, {(1, 3, 3): 1}), 4, 4, 2)
    want = leafset(sc.uniform(4, 4)) - {(0, 1, 1), (0, 2, 1), (0, 1, 2), (0, 2, 2)}
    want |= {(1, 2, 2), (1, 3, 2), (1, 2, 3)}
    want |= {(2, 6 + a, 6 + b) for a in (0, 1) for b in (0, 1)}
    for (x, y) in ((2, 1), (1, 2), (2, 2)):
        want |= {(1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1)}
    assert out == want
    assert len(out) == 31 and adapt.is_balanced(out, 4, 4)


def test_merge_and_blocked_merge():
    base = leafset(sc.uniform(4, 4)) - {(0, 1, 1), (0, 2, 1), (0, 1, 2), (0, 2, 2)}
    base |= {(1, 2, 2), (1, 3, 2), (1, 2, 3)}
    base |= {(2, 6 + a, 6 + b) for a in (0, 1) for b in (0, 1)}
    for (x, y) in ((2, 1), (1, 2), (2, 2)):
        base |= {(1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1)}
    cols = sorted(base)
    lvl2 = {(2, 6 + a, 6 + b): -1 for a in (0, 1) for b in (0, 1)}
    east = {(1, 4 + a, 2 + b): -1 for a in (0, 1) for b in (0, 1)}
    # the level-2 family merges back into (1,3,3)
    out = adapt.adapt_columns(cols, flags_for(cols, lvl2), 4, 4, 2)
    assert out == (base - set(lvl2)) | {(1, 3, 3)}
    # the east family touches level-2 leaves: blocked, even when the level-2
    # family merges in the same pass (merges are decided on one layout)
    out = adapt.adapt_columns(cols, flags_for(cols, east), 4, 4, 2)
    assert out == base
    out = adapt.adapt_columns(cols, flags_for(cols, {**lvl2, **east}), 4, 4, 2)
    assert out == (base - set(lvl2)) | {(1, 3, 3)}
    # an incomplete family never merges
    part = dict(list(lvl2.items())[:3])
    assert adapt.adapt_columns(cols, flags_for(cols, part), 4, 4, 2) == base


def random_layout(seed, nx0, ny0, lvl_max, periodic=True):
    rng = np.random.default_rng(seed)
    marks = {}

    def tgt(l, x, y):
        key = (l, x, y)
        if key not in marks:
            marks[key] = rng.random() < 0.3
        return l + 1 if marks[key] else l
    return sc.refine_to_target(nx0, ny0, tgt, lvl_max, periodic)


@pytest.mark.parametrize("seed", range(12))
def test_random_layout_invariants(seed):
    rng = np.random.default_rng(100 + seed)
    periodic = seed % 3 != 2
    nx0, ny0, lvl_max = 4, 3, 3
    cols = random_layout(seed, nx0, ny0, lvl_max - 1, periodic)
    old = leafset(cols)
    flags = rng.choice(np.array([-1, 0, 1], np.int8), size=len(cols), p=[0.4, 0.4, 0.2])
    out = adapt.adapt_columns(cols, flags, nx0, ny0, lvl_max, periodic, periodic)
    assert covers(out, nx0, ny0)
    assert adapt.is_balanced(out, nx0, ny0, periodic, periodic)
    fl = {c: int(f) for c, f in zip(map(tuple, np.asarray(cols).tolist()), flags)}
    for (l, x, y), f in fl.items():
        if f == 1 and l < lvl_max:
            assert (l, x, y) not in out and adapt._leaf_over(out, l, x, y) is None
    for (l, x, y) in out - old:
        if any((l + 1, 2 * x + a, 2 * y + b) in old for a in (0, 1) for b in (0, 1)):
            kids = [(l + 1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1)]
            assert all(fl.get(k) == -1 for k in kids)


@pytest.mark.parametrize("seed", range(8))
def test_balance_splits_are_minimal(seed):
    """With no merges, every split not asked for was forced: the parent box of
    such a leaf touches a leaf two levels finer than the parent."""
    rng = np.random.default_rng(200 + seed)
    nx0, ny0, lvl_max = 4, 4, 3
    cols = random_layout(seed, nx0, ny0, 2)
    flags = (rng.random(len(cols)) < 0.25).astype(np.int8)
    out = adapt.adapt_columns(cols, flags, nx0, ny0, lvl_max)
    asked = set()
    for (l, x, y), f in zip(map(tuple, np.asarray(cols).tolist()), flags):
        asked.add((l, x, y))
        if f == 1 and l < lvl_max:
            asked |= {(l + 1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1)}
    depth = max(l for l, _, _ in out)
    lmap = adapt.finest_level_map(out, nx0, ny0, depth)
    for (l, x, y) in out - asked:
        p = (l - 1, x >> 1, y >> 1)
        assert adapt.ring_max_level(lmap, *p, depth, True, True) >= p[0] + 2


# ------------------------------------------------------------------ transfer
def omesh(cols, N=4, periodic=True, nx0=4, ny0=4, n_z=2):
    cols = sc.morton_sort(np.array(sorted(leafset(cols))), 4)
    return OracleMesh(N, nx0, ny0, 400e3, 400e3, np.linspace(0, 20e3, n_z + 1), cols,
                      periodic, periodic)


def _poly(xyz, N):
    x, y, z = xyz[:, 0] / 4e5, xyz[:, 1] / 4e5, xyz[:, 2] / 2e4
    return (1 + x - 0.7 * x**N) * (0.5 - y**N + 0.2 * y**2) + 0.3 * x**(N - 1) * y * z**N


def test_transfer_identity():
    m = omesh(random_layout(1, 4, 4, 2))
    q = np.random.default_rng(0).standard_normal((2, m.n_dof))
    np.testing.assert_array_equal(adapt.transfer(m, m, q), q)


def family_flags(cols, rng, p_merge=0.5, p_split=0.2):
    """-1 on whole sibling families (probability p_merge each), +1 on other
    columns with probability p_split."""
    cs = [tuple(int(t) for t in c) for c in np.asarray(cols).reshape(-1, 3)]
    have = set(cs)
    out = {}
    for (l, x, y) in cs:
        if l == 0 or (x & 1) or (y & 1):
            continue
        fam = [(l, x + a, y + b) for a in (0, 1) for b in (0, 1)]
        if all(f in have for f in fam) and rng.random() < p_merge:
            out.update({f: -1 for f in fam})
    for c in cs:
        if c not in out and rng.random() < p_split:
            out[c] = 1
    return flags_for(cols, out)


@pytest.mark.parametrize("seed,N", [(0, 3), (1, 4), (2, 5), (3, 4)])
def test_transfer_reproduces_polynomials(seed, N):
    rng = np.random.default_rng(300 + seed)
    cols = random_layout(seed, 4, 4, 2, periodic=False)
    flags = family_flags(cols, rng, 0.9, 0.1)
    new = adapt.adapt_columns(cols, flags, 4, 4, 3, False, False)
    kinds = {k for k, _ in adapt.classify(np.array(sorted(leafset(cols))), np.array(sorted(new)))}
    assert kinds == {"same", "child", "parent"}
    a, b = omesh(cols, N, False), omesh(new, N, False)
    q = adapt.transfer(a, b, _poly(a.node_xyz, N)[None])
    want = _poly(b.node_xyz, N)
    assert np.max(np.abs(q[0] - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("seed,N", [(0, 4), (1, 3), (2, 7)])
def test_split_then_merge_round_trip(seed, N):
    rng = np.random.default_rng(400 + seed)
    cols = random_layout(seed, 4, 4, 1)
    lvl0 = [c for c in map(tuple, np.asarray(cols).tolist()) if c[0] == 0]
    pick = {c: 1 for c in lvl0 if rng.random() < 0.5}
    mid = adapt.adapt_columns(cols, flags_for(cols, pick), 4, 4, 2)
    made = {(1, 2 * x + a, 2 * y + b): -1 for (_, x, y) in pick for a in (0, 1) for b in (0, 1)}
    mid_cols = sorted(mid)
    back = adapt.adapt_columns(mid_cols, flags_for(mid_cols, made), 4, 4, 2)
    assert back == leafset(cols)
    a, b = omesh(cols, N), omesh(mid, N)
    q = rng.standard_normal((3, a.n_dof))
    q2 = adapt.transfer(b, a, adapt.transfer(a, b, q))
    assert np.max(np.abs(q2 - q)) <= 1e-12


def test_transfer_conserves_mass():
    rng = np.random.default_rng(7)
    # splits on a two-level layout
    cols = random_layout(5, 4, 4, 1)
    pick = {c: 1 for c in map(tuple, np.asarray(cols).tolist()) if rng.random() < 0.4}
    new = adapt.adapt_columns(cols, flags_for(cols, pick), 4, 4, 2)
    a, b = omesh(cols), omesh(new)
    q = rng.standard_normal((2, a.n_dof))
    q2 = adapt.transfer(a, b, q)
    for f in range(2):
        s0, s1 = a.MG @ q[f], b.MG @ q2[f]
        assert abs(s1 - s0) <= 1e-12 * (a.MG @ np.abs(q[f]))
    # merging every family of a uniform level-1 layout
    fine = sc.uniform(8, 8)
    fine[:, 0] = 1
    fine_cols = np.array([(1, x, y) for (_, x, y) in fine])
    allm = adapt.adapt_columns(fine_cols, -np.ones(len(fine_cols), np.int8), 4, 4, 1)
    assert allm == leafset(sc.uniform(4, 4))
    a, b = omesh(fine_cols), omesh(allm)
    q = rng.standard_normal((2, a.n_dof))
    q2 = adapt.transfer(a, b, q)
    for f in range(2):
        s0, s1 = a.MG @ q[f], b.MG @ q2[f]
        assert abs(s1 - s0) <= 1e-12 * (a.MG @ np.abs(q[f]))


def test_unweighted_projection_would_fail_conservation():
    """The weighting matters: a projection without the lumped masses (a
    plausible slip) breaks the conservation pin above."""
    rng = np.random.default_rng(8)
    fine_cols = np.array([(1, x, y) for x in range(8) for y in range(8)])
    allm = adapt.adapt_columns(fine_cols, -np.ones(64, np.int8), 4, 4, 1)
    a, b = omesh(fine_cols), omesh(allm)
    q = rng.standard_normal((1, a.n_dof))
    orig = a.mL.copy()
    try:
        a.mL = np.ones_like(orig)
        q2 = adapt.transfer(a, b, q)
    finally:
        a.mL = orig
    assert abs(b.MG @ q2[0] - a.MG @ q[0]) > 1e-6 * (a.MG @ np.abs(q[0]))
