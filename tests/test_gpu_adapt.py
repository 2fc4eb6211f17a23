"""GPU tests of dynamic adaptation: the transfer kernel against the oracle's
element-wise transfer, and a whole adaptive run (flags -> new layout ->
transfer -> RK3 stages, repeated) against the same sequence computed by the
oracle."""

import sys

import numpy as np
import pytest

from harness import match, oracle_mesh, oracle_reference_local
from oracle import adapt, amr, assembly, metrics, timestep
from synth import cases
from synth import columns as sc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def case_with(cols, N, periodic):
    c = cases.get("small_amr3", N=N, periodic=periodic)
    c["columns"] = np.asarray(cols, dtype=np.int64)
    return c


@pytest.mark.parametrize("seed,N,periodic", [(0, 4, True), (1, 7, True), (2, 3, False), (3, 5, True)])
def test_transfer_kernel_matches_oracle(seed, N, periodic):
    import torch
    from paper_2410_21607_amd import api
    say("transfer", seed, N, periodic)
    rng = np.random.default_rng(70 + seed)
    a_cols = random_layout(seed, 4, 4, 2, periodic)
    ca = case_with(a_cols, N, periodic)
    ga = api.Mesh.from_case(ca)
    b_cols = api.sem_adapt_columns(ga, a_cols, family_flags(a_cols, rng), 3)
    cb = case_with(b_cols, N, periodic)
    gb = ga.with_columns(b_cols)
    oa, ob = oracle_mesh(ca), oracle_mesh(cb)
    pa = match(oa.node_xyz, ga.node_xyz(), ca)
    pb = match(ob.node_xyz, gb.node_xyz(), cb)
    q = rng.standard_normal((5, oa.n_dof))
    T = api.Transfer(ga, gb)
    out = torch.full((gb.n_state,), float("nan"), dtype=torch.float64, device="cuda")
    api.sem_transfer_apply(T, ga.unpack(q[:, pa]), out)
    torch.cuda.synchronize()
    pad = out.reshape(5, gb.info["n_h"], gb.ldz)[:, :, gb.info["nzn"]:]
    assert torch.all(pad == 0)
    got = np.empty((5, ob.n_dof))
    got[:, pb] = gb.pack(out)
    want = adapt.transfer(oa, ob, q)
    err = np.max(np.abs(got - want))
    say("  max abs err", err)
    assert err <= 1e-13 * np.max(np.abs(want))


def _oracle_adaptive(c, q, lvl_max, thr, interval, n_steps, criterion=1):
    """The same adaptive sequence on the oracle: RK3 steps, then every
    `interval` steps criterion flags (1: vertical vorticity, 0: wind speed)
    -> new layout -> transfer."""
    cols = np.asarray(c["columns"])
    om = oracle_mesh(c)
    steps = 0
    layouts = []
    while steps < n_steps:
        ref = oracle_reference_local(c, om)
        q, _ = timestep.run_stages(lambda s: assembly.rhs(om, s, ref, c["phys"]), q, c["dt"],
                                   3 * interval)
        steps += interval
        qL = assembly.scatter(om, q)
        C = amr.criterion_vorticity(om, qL) if criterion == 1 else amr.criterion_speed(qL)
        ef = amr.element_flags(C.reshape(om.n_elem, -1), om.e_level, thr, lvl_max)
        cf = amr.column_flags(ef, om.columns, om.n_z)
        new = adapt.adapt_columns(om.columns, cf, c["nx0"], c["ny0"], lvl_max,
                                  c["periodic_x"], c["periodic_y"])
        cmax = C.reshape(om.n_elem, -1).max(axis=1)
        layouts.append((new, cmax))
        if new != {tuple(int(t) for t in r) for r in om.columns}:
            c = dict(c, columns=sc.morton_sort(np.array(sorted(new)), lvl_max))
            nm = oracle_mesh(c)
            q = adapt.transfer(om, nm, q)
            om = nm
    return c, om, q, layouts


def test_adaptive_run_matches_oracle():
    import torch
    from paper_2410_21607_amd import api
    from paper_2410_21607_amd.adaptive import AdaptiveRun
    c = cases.get("small_amr2", N=4)
    lvl_max, thr, interval, n_steps = 2, [1.5e-4, 3.5e-4], 2, 6
    say("adaptive run", c["name"], "thr", thr)
    gm = api.Mesh.from_case(c)
    _, _, z = gm.coords()
    bg = cases.reference_state(c, z)
    ref = (bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    gm.set_reference(*ref)
    om = oracle_mesh(c)
    perm = match(om.node_xyz, gm.node_xyz(), c)
    q_or = cases.initial_state(c, om.node_xyz)
    run = AdaptiveRun(gm, gm.unpack(q_or[:, perm]), c["dt"], ref, api.SEM_CRIT_VORTZ, thr,
                      lvl_max, interval, graph=True)
    run.run(n_steps)
    torch.cuda.synchronize()
    c2, om2, want, layouts = _oracle_adaptive(c, q_or, lvl_max, thr, interval, n_steps)
    # the thresholds must sit away from every element maximum, or round-off
    # could legitimately flip a flag
    for _, cmax in layouts:
        for t in thr:
            assert np.min(np.abs(cmax - t)) > 1e-9 * t
    say("  rebuilds", run.n_rebuild, "history", run.history)
    assert run.n_rebuild >= 1
    got_cols = {tuple(int(t) for t in r) for r in run.mesh.columns}
    assert got_cols == {tuple(int(t) for t in r) for r in om2.columns}
    p2 = match(om2.node_xyz, run.mesh.node_xyz(), c2)
    got = np.empty_like(want)
    got[:, p2] = run.mesh.pack(run.q)
    err = metrics.rel_l2(got, want, metrics.STATE_FLOORS)
    say("  rel", err)
    assert err.max() <= 1e-12


def test_adaptive_run_speed_criterion_matches_oracle():
    """The paper's criterion, the wind speed |u| at every node against one
    threshold per level, driving the whole adaptive loop (flags -> layout ->
    transfer -> stages) on a vortex moved by a steering wind, three levels:
    the GPU run ends on the oracle's layout with the oracle's state."""
    import torch
    from paper_2410_21607_amd import api
    from paper_2410_21607_amd.adaptive import AdaptiveRun
    c = cases.get("small_amr2", N=4)
    c["steer"] = (6.0, -4.0)
    lvl_max, interval, n_steps = 3, 2, 6
    say("adaptive run, speed criterion", c["name"])
    gm = api.Mesh.from_case(c)
    _, _, z = gm.coords()
    bg = cases.reference_state(c, z)
    ref = (bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    gm.set_reference(*ref)
    om = oracle_mesh(c)
    perm = match(om.node_xyz, gm.node_xyz(), c)
    q_or = cases.initial_state(c, om.node_xyz)
    # thresholds between the element maxima of |u| of the initial state,
    # in wide gaps so that the drift of later boundaries cannot reach them
    C0 = amr.criterion_speed(assembly.scatter(om, q_or)).reshape(om.n_elem, -1).max(axis=1)
    v = np.sort(C0)
    gaps = np.diff(v)
    cand = np.argsort(gaps)[::-1][:8]
    cuts = sorted(0.5 * (v[i] + v[i + 1]) for i in cand if v[i] > v[0] + 0.25 * (v[-1] - v[0]))
    thr = [cuts[0], cuts[len(cuts) // 2], cuts[-1]]
    run = AdaptiveRun(gm, gm.unpack(q_or[:, perm]), c["dt"], ref, api.SEM_CRIT_SPEED, thr,
                      lvl_max, interval, graph=True)
    run.run(n_steps)
    torch.cuda.synchronize()
    c2, om2, want, layouts = _oracle_adaptive(c, q_or, lvl_max, thr, interval, n_steps, criterion=0)
    for _, cmax in layouts:
        for t in thr:
            assert np.min(np.abs(cmax - t)) > 1e-9 * t
    say("  thresholds", thr, "rebuilds", run.n_rebuild, "history", run.history)
    assert run.n_rebuild >= 1
    assert max(int(r[0]) for r in run.mesh.columns) >= 2
    got_cols = {tuple(int(t) for t in r) for r in run.mesh.columns}
    assert got_cols == {tuple(int(t) for t in r) for r in om2.columns}
    p2 = match(om2.node_xyz, run.mesh.node_xyz(), c2)
    got = np.empty_like(want)
    got[:, p2] = run.mesh.pack(run.q)
    err = metrics.rel_l2(got, want, metrics.STATE_FLOORS)
    say("  rel", err)
    assert err.max() <= 1e-12
