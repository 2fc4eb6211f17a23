"""CPU checks of the host-only adaptation calls of the C ABI against the
oracle: the adapted column layout (integer work: the same set of columns,
bit for bit) and the solution-transfer rows (applied on the host to random
fields and compared with the oracle's element-wise transfer)."""

import os

import numpy as np
import pytest

from oracle import adapt
from oracle.mesh import OracleMesh
from synth import columns as sc

from harness import match

native = pytest.importorskip("paper_2410_21607_amd.native")


def _lib():
    if not os.path.exists(native.LIB_PATH):
        pytest.skip("libsem.so not built")
    return native.lib()


def params(N=4, periodic=True, nx0=4, ny0=4, n_z=2):
    return dict(N=N, nx0=nx0, ny0=ny0, Lx=400e3, Ly=400e3 * ny0 / nx0,
                z_edges=np.linspace(0.0, 20e3, n_z + 1), periodic_x=periodic,
                periodic_y=periodic, f=5e-5, g=9.81, R_d=287.0, c_p=1004.0, p00=1e5)


def random_layout(seed, nx0, ny0, lvl_max, periodic=True):
    rng = np.random.default_rng(seed)
    marks = {}

    def tgt(l, x, y):
        if (l, x, y) not in marks:
            marks[(l, x, y)] = rng.random() < 0.3
        return l + 1 if marks[(l, x, y)] else l
    return sc.refine_to_target(nx0, ny0, tgt, lvl_max, periodic)


def family_flags(cols, rng, p_merge=0.6, p_split=0.15):
    cs = [tuple(int(t) for t in c) for c in np.asarray(cols)]
    have = set(cs)
    out = {}
    for (l, x, y) in cs:
        if l and not (x & 1) and not (y & 1):
            fam = [(l, x + a, y + b) for a in (0, 1) for b in (0, 1)]
            if all(f in have for f in fam) and rng.random() < p_merge:
                out.update({f: -1 for f in fam})
    for c in cs:
        if c not in out and rng.random() < p_split:
            out[c] = 1
    return np.array([out.get(c, 0) for c in cs], np.int8)


def as_set(cols):
    return {tuple(int(t) for t in c) for c in np.asarray(cols).reshape(-1, 3)}


@pytest.mark.parametrize("seed", range(16))
def test_adapt_columns_matches_oracle(seed):
    _lib()
    from paper_2410_21607_amd import api
    rng = np.random.default_rng(seed)
    periodic = seed % 4 != 3
    nx0, ny0 = (4, 4) if seed % 2 else (5, 3)
    lvl_max = 3
    cols = random_layout(seed, nx0, ny0, 2, periodic)
    if seed % 3 == 0:
        flags = rng.choice(np.array([-1, 0, 1], np.int8), size=len(cols))
    else:
        flags = family_flags(cols, rng)
    p = params(periodic=periodic, nx0=nx0, ny0=ny0)
    got = api.sem_adapt_columns(p, cols, flags, lvl_max)
    want = adapt.adapt_columns(cols, flags, nx0, ny0, lvl_max, periodic, periodic)
    assert as_set(got) == want
    assert len(got) == len(want)
    # Morton order of the finest level present (a valid order; the set is what is unique)
    assert np.array_equal(got, sc.morton_sort(got, int(got[:, 0].max())))


def test_adapt_columns_errors():
    _lib()
    from paper_2410_21607_amd import api
    p = params()
    cols = sc.uniform(4, 4)
    bad = np.concatenate([cols, [[1, 0, 0]]])          # overlaps (0,0,0)
    with pytest.raises(native.SemError):
        api.sem_adapt_columns(p, bad, np.zeros(len(bad), np.int8), 2)
    with pytest.raises(native.SemError):
        api.sem_adapt_columns(p, cols[:-1], np.zeros(len(cols) - 1, np.int8), 2)   # gap
    with pytest.raises(native.SemError):
        api.sem_adapt_columns(p, cols, np.zeros(len(cols), np.int8), 99)


def _oracle_mesh(p, cols):
    return OracleMesh(p["N"], p["nx0"], p["ny0"], p["Lx"], p["Ly"], p["z_edges"], cols,
                      p["periodic_x"], p["periodic_y"])


def _apply_rows(ptr, src, w, qh, n_to):
    """q_to[h] = sum w q_from[src] for a (F, n_h_from, nzn) array."""
    out = np.zeros((qh.shape[0], n_to, qh.shape[2]))
    for h in range(n_to):
        for r in range(ptr[h], ptr[h + 1]):
            out[:, h, :] += w[r] * qh[:, src[r], :]
    return out


@pytest.mark.parametrize("seed,N,periodic", [(0, 4, True), (1, 3, True), (2, 5, False),
                                             (3, 4, False), (4, 7, True), (5, 2, True)])
def test_transfer_rows_match_oracle(seed, N, periodic):
    _lib()
    from paper_2410_21607_amd import api
    rng = np.random.default_rng(50 + seed)
    p = params(N=N, periodic=periodic)
    case = dict(Lx=p["Lx"], Ly=p["Ly"], periodic_x=periodic, periodic_y=periodic)
    a_cols = random_layout(seed, 4, 4, 2, periodic)
    flags = family_flags(a_cols, rng)
    b_cols = api.sem_adapt_columns(p, a_cols, flags, 3)
    ptr, src, w = api.sem_transfer_plan(p, a_cols, b_cols)
    pa, pb = api.sem_mesh_plan(dict(p, columns=a_cols, phys=p)), \
        api.sem_mesh_plan(dict(p, columns=b_cols, phys=p))
    oa, ob = _oracle_mesh(p, a_cols), _oracle_mesh(p, b_cols)
    kinds = {k for k, _ in adapt.classify(oa.columns, ob.columns)}
    assert kinds == {"same", "child", "parent"}
    nzn = pa[3].size

    def gxyz(plan):
        hxy, z = plan[1], plan[3]
        return np.column_stack([np.repeat(hxy[:, 0], nzn), np.repeat(hxy[:, 1], nzn),
                                np.tile(z, len(hxy))])
    perm_a = match(oa.node_xyz, gxyz(pa), case)     # library order -> oracle index
    perm_b = match(ob.node_xyz, gxyz(pb), case)
    q_or = rng.standard_normal((3, oa.n_dof))
    q_lib = q_or[:, perm_a].reshape(3, -1, nzn)
    got = _apply_rows(ptr, src, w, q_lib, len(ptr) - 1).reshape(3, -1)
    want = adapt.transfer(oa, ob, q_or)[:, perm_b]
    err = np.max(np.abs(got - want))
    assert err <= 1e-13 * np.max(np.abs(want)), err


@pytest.mark.parametrize("seed", range(6))
def test_forecast_labels_match_oracle(seed):
    """Training classes (integer work): bit-exact against the oracle on a
    layout and its adapted successor, with random levels asked for."""
    _lib()
    from paper_2410_21607_amd import api
    from oracle import forecast
    rng = np.random.default_rng(90 + seed)
    p = params(n_z=3)
    at = random_layout(seed, 4, 4, 2)
    later = api.sem_adapt_columns(p, at, family_flags(at, rng, 0.5, 0.3), 3)
    dem = rng.integers(0, 4, size=len(later) * 3).astype(np.int8)
    got = api.sem_forecast_labels(p, at, later, dem)
    want = forecast.labels(at, later, dem, 3)
    np.testing.assert_array_equal(got, want)
    # and the other way round (a later layout coarser in places)
    dem2 = rng.integers(0, 4, size=len(at) * 3).astype(np.int8)
    np.testing.assert_array_equal(api.sem_forecast_labels(p, later, at, dem2),
                                  forecast.labels(later, at, dem2, 3))


def test_transfer_plan_rejects_unrelated_layouts():
    """A column more than one level away from every old column, or meshes
    with different orders, are rejected before any work."""
    _lib()
    from paper_2410_21607_amd import api
    p = params()
    a = sc.uniform(4, 4)
    b = np.array([(2, x, y) for x in range(16) for y in range(16)])   # two levels finer
    with pytest.raises(native.SemError):
        api.sem_transfer_plan(p, a, b)


def test_forecast_labels_reject_mismatched_layouts():
    _lib()
    from paper_2410_21607_amd import api
    p = params(n_z=2)
    a = sc.uniform(4, 4)
    with pytest.raises(ValueError):
        api.sem_forecast_labels(p, a, a, np.zeros(3, np.int8))     # wrong dem size
    q = dict(p, nx0=5)
    with pytest.raises(native.SemError):
        api.sem_forecast_labels(q, sc.uniform(5, 4), a, np.zeros(len(a) * 2, np.int8))


def test_same_layout_compares_column_sets():
    """The adaptive loop's unchanged-layout check: the same (level, ix, iy)
    set in any order is the same layout; one column more, or one index
    changed, is not."""
    from paper_2410_21607_amd.adaptive import _same_layout
    a = np.asarray(random_layout(5, 4, 4, 3), dtype=np.int32)
    perm = np.random.default_rng(1).permutation(len(a))
    assert _same_layout(a, a[perm])
    assert not _same_layout(a, a[:-1])
    b = a.copy()
    b[len(b) // 2, 2] += 1
    assert not _same_layout(a, b)
    c = a.copy()
    c[[0, 1]] = c[[1, 0]]
    c[0, 0], c[1, 0] = c[1, 0], c[0, 0]   # swap levels only: a different set unless equal
    assert _same_layout(a, c) == (set(map(tuple, a.tolist())) == set(map(tuple, c.tolist())))
