"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded
inputs (uniform, two-level and three-level meshes, N from 3 to 8, ragged
element counts).  Bar: floor-scaled relative L2 <= 1e-12 per field in FP64;
bit-exact refinement flags."""

import sys

import numpy as np
import pytest

from harness import _keys, match, oracle_mesh, oracle_reference_local
from oracle import amr as oamr
from oracle import assembly, euler, metrics, timestep
from synth import cases

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

CASES = [("vortex_8x8x4_n4", {}), ("small_uniform", {"N": 3}), ("small_amr2", {}),
         ("small_amr2", {"N": 7}), ("small_amr3", {}), ("small_amr3", {"N": 7}),
         ("small_amr2", {"N": 8}), ("small_amr3", {"N": 5, "periodic": False})]
IDS = [f"{n}-{'-'.join(f'{k}{v}' for k, v in kw.items())}" for n, kw in CASES]

_CACHE = {}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Setup:
    def __init__(self, name, kw):
        import torch
        from paper_2410_21607_amd import api
        self.torch, self.api = torch, api
        self.c = c = cases.get(name, **dict(kw))
        self.gm = api.Mesh.from_case(c)
        hxy, hhxy, z = self.gm.coords()
        bg = cases.reference_state(c, z)
        self.gm.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
        self.om = oracle_mesh(c)
        self.gxyz = self.gm.node_xyz()
        self.perm = match(self.om.node_xyz, self.gxyz, c)
        self.q_or = cases.initial_state(c, self.om.node_xyz)
        # the synthetic field evaluated at the GPU's own node positions agrees
        # to round-off; the parity runs feed both sides bit-identical values
        # (the oracle-position field permuted into the GPU numbering), since
        # the right-hand side amplifies ulp-level input differences through
        # the hydrostatic and gradient-wind cancellations
        q_g = cases.initial_state(c, self.gxyz)
        np.testing.assert_allclose(q_g, self.q_or[:, self.perm], rtol=1e-12, atol=1e-12)
        self.q_g = self.gm.unpack(self.q_or[:, self.perm])
        self.ref = oracle_reference_local(c, self.om)

    def to_oracle_order(self, flat):
        a = self.gm.pack(flat)
        out = np.empty_like(a)
        out[:, self.perm] = a
        return out


def get(name, kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = Setup(name, kw)
    return _CACHE[key]


@pytest.mark.parametrize("name,kw", CASES, ids=IDS)
def test_nc_scatter(name, kw):
    S = get(name, kw)
    if S.gm.n_hang == 0:
        pytest.skip("conforming mesh")
    torch, api = S.torch, S.api
    say("nc_scatter", name, kw)
    hv = torch.zeros(S.gm.n_hstate, dtype=torch.float64, device="cuda")
    api.sem_nc_project(S.gm, api.SEM_SCATTER, S.q_g, hv)
    torch.cuda.synchronize()
    qL = assembly.scatter(S.om, S.q_or).reshape(5, -1)
    oh = np.column_stack([S.om.xl.ravel(), S.om.yl.ravel(), S.om.zl.ravel()])[S.om.hanging]
    _, first = np.unique(_keys(oh, S.c), axis=0, return_index=True)
    hidx = np.nonzero(S.om.hanging)[0][first]
    perm = match(oh[first], S.gm.hang_xyz(), S.c)
    got = S.gm.pack_hang(hv)
    want = qL[:, hidx][:, perm]
    err = metrics.rel_l2(got, want, metrics.STATE_FLOORS)
    say("  rel", err)
    assert err.max() <= TOL64


def _element_contrib(S):
    """Oracle m_L R_L in element/local order (E, (N+1)^3) per field."""
    qL = assembly.scatter(S.om, S.q_or)
    RL = euler.element_rhs(S.om, qL, S.ref["rho0"], S.ref["theta0"], S.ref["dtheta0dz"],
                           S.c["phys"])
    return RL.reshape(5, -1) * S.om.mL[None, :]


@pytest.mark.parametrize("name,kw", CASES, ids=IDS)
def test_rhs_element_contributions(name, kw):
    S = get(name, kw)
    torch, api = S.torch, S.api
    say("sem_rhs", name, kw)
    hv = torch.zeros(S.gm.n_hstate, dtype=torch.float64, device="cuda")
    if S.gm.n_hang:
        api.sem_nc_project(S.gm, api.SEM_SCATTER, S.q_g, hv)
    rE = torch.zeros(5 * S.gm.n_local, dtype=torch.float64, device="cuda")
    api.sem_rhs(S.gm, S.q_g, hv if S.gm.n_hang else None, rE, api.SEM_FP64)
    torch.cuda.synchronize()
    want = _element_contrib(S)
    got = rE.cpu().numpy().reshape(5, -1)
    floors = metrics.RHS_FLOORS * S.om.mL.mean()
    err = metrics.rel_l2(got, want, floors)
    say("  rel", err)
    assert err.max() <= TOL64


def _gpu_rhs(S, prec):
    torch, api = S.torch, S.api
    n, nh, nl = S.gm.n_state, S.gm.n_hstate, 5 * S.gm.n_local
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda")
    hv, rE, acc, cH, r = z(nh), z(nl), z(n), z(nh), z(n)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_SCATTER, S.q_g, hv)
    api.sem_rhs(S.gm, S.q_g, hv if nh else None, rE, prec)
    api.sem_dss(S.gm, api.SEM_ASSEMBLE, rE=rE, acc=acc, c=cH if nh else None)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_GATHER, cH, acc)
    api.sem_dss(S.gm, api.SEM_FINALIZE, acc=acc, r=r)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("name,kw", CASES, ids=IDS)
def test_full_rhs_through_dss(name, kw):
    S = get(name, kw)
    say("rhs+dss", name, kw)
    r = _gpu_rhs(S, S.api.SEM_FP64)
    want = assembly.rhs(S.om, S.q_or, S.ref, S.c["phys"])
    err = metrics.rel_l2(S.to_oracle_order(r), want, metrics.RHS_FLOORS)
    say("  rel", err)
    assert err.max() <= TOL64


@pytest.mark.parametrize("name,kw", CASES[:3] + CASES[4:6], ids=IDS[:3] + IDS[4:6])
def test_fp32_rhs_error(name, kw):
    """FP32 element arithmetic against the FP64 oracle, floor-scaled."""
    S = get(name, kw)
    say("rhs fp32", name, kw)
    r = _gpu_rhs(S, S.api.SEM_FP32)
    want = assembly.rhs(S.om, S.q_or, S.ref, S.c["phys"])
    err = metrics.rel_l2(S.to_oracle_order(r), want, metrics.RHS_FLOORS)
    say("  rel fp32", err)
    assert err.max() <= 1e-4


@pytest.mark.parametrize("name,kw", CASES, ids=IDS)
def test_stages_match_oracle(name, kw):
    S = get(name, kw)
    torch, api = S.torch, S.api
    nst = S.c["stages"]
    dt = S.c["dt"]
    say("stages", name, kw, nst)
    qn = S.q_g.clone()
    qs = S.q_g.clone()
    out = torch.zeros_like(qn)
    for st in range(nst):
        a, b, cc = timestep.stage_coefficients(st % 3, dt)
        api.sem_stage(S.gm, a, b, cc, qn, qs, out, api.SEM_FP64)
        qs, out = out, qs
        if st % 3 == 2:
            qn.copy_(qs)
    torch.cuda.synchronize()
    rhs = lambda q: assembly.rhs(S.om, q, S.ref, S.c["phys"])
    want, _ = timestep.run_stages(rhs, S.q_or, dt, nst)
    err = metrics.rel_l2(S.to_oracle_order(qs), want, metrics.STATE_FLOORS)
    say("  rel", err)
    assert err.max() <= TOL64


@pytest.mark.parametrize("alias", ["none", "qout=qs", "qout=qn", "qout=r"])
def test_stage_update_matches_oracle(alias):
    """sem_stage_update against oracle.timestep.stage_update on the same
    seeded arrays, every entry including the row padding, for each of the
    three SSP-RK3 stages; the call allows its output to alias any input."""
    S = get(*CASES[0])
    torch, api = S.torch, S.api
    say("stage_update", alias)
    n = S.gm.n_state
    rng = np.random.default_rng(11)
    for st in range(3):
        a, b, cc = timestep.stage_coefficients(st, S.c["dt"])
        qn, qs, r = (rng.standard_normal(n) for _ in range(3))
        want = timestep.stage_update(a, b, cc, qn, qs, r)
        dqn, dqs, dr = (torch.from_numpy(v.copy()).cuda() for v in (qn, qs, r))
        out = {"none": torch.zeros_like(dqn), "qout=qs": dqs, "qout=qn": dqn, "qout=r": dr}[alias]
        api.sem_stage_update(S.gm, a, b, cc, dqn, dqs, dr, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # one fused multiply-add chain against numpy's separate roundings
        np.testing.assert_allclose(got, want, rtol=4e-16, atol=4e-16 * np.abs(want).max())


def _unfused_stage(S, a, b, cc, qn, qs):
    """q_out by the per-step calls: scatter, element right-hand side,
    assemble, gather, finalize, stage update."""
    torch, api = S.torch, S.api
    n, nh, nl = S.gm.n_state, S.gm.n_hstate, 5 * S.gm.n_local
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda")
    hv, rE, acc, cH, r, out = z(nh), z(nl), z(n), z(nh), z(n), z(n)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_SCATTER, qs, hv)
    api.sem_rhs(S.gm, qs, hv if nh else None, rE, api.SEM_FP64)
    api.sem_dss(S.gm, api.SEM_ASSEMBLE, rE=rE, acc=acc, c=cH if nh else None)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_GATHER, cH, acc)
    api.sem_dss(S.gm, api.SEM_FINALIZE, acc=acc, r=r)
    api.sem_stage_update(S.gm, a, b, cc, qn, qs, r, out)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("name,kw", CASES, ids=IDS)
def test_fused_stage_equals_unfused_composition(name, kw):
    """sem_stage against the composition of the per-step calls on the same
    input: the stage output of each of the three SSP-RK3 stages within 1e-14
    relative (floor-scaled), and the bare right-hand side ((a, b, c) =
    (0, 0, 1)) within 1e-13, the two paths summing the same contributions in
    different orders."""
    S = get(name, kw)
    torch, api = S.torch, S.api
    say("fused vs unfused", name, kw)
    dt = S.c["dt"]
    rng = np.random.default_rng(3)
    qn_h = S.gm.pack(S.q_g)
    # q_s: the workload's state with a relative perturbation of every field,
    # so that q^n and q_s differ and a, b and c all matter
    qs_h = qn_h * (1.0 + 1e-3 * rng.standard_normal(qn_h.shape))
    qn, qs = S.gm.unpack(qn_h), S.gm.unpack(qs_h)
    for st, (a, b, cc) in enumerate([timestep.stage_coefficients(k, dt) for k in range(3)]
                                    + [(0.0, 0.0, 1.0)]):
        fused = torch.zeros_like(qn)
        api.sem_stage(S.gm, a, b, cc, qn, qs, fused, api.SEM_FP64)
        unf = _unfused_stage(S, a, b, cc, qn, qs)
        floors = metrics.STATE_FLOORS if st < 3 else metrics.RHS_FLOORS
        err = metrics.rel_l2(S.gm.pack(fused), S.gm.pack(unf), floors)
        say("  stage" if st < 3 else "  rhs", st, "rel", err)
        assert err.max() <= (1e-14 if st < 3 else 1e-13)


@pytest.mark.parametrize("name,kw", [CASES[0], CASES[2], CASES[4], CASES[5]],
                         ids=[IDS[0], IDS[2], IDS[4], IDS[5]])
@pytest.mark.parametrize("criterion", [0, 1])
def test_amr_flag_bit_exact(name, kw, criterion):
    S = get(name, kw)
    torch, api = S.torch, S.api
    say("amr_flag", name, kw, criterion)
    qL = assembly.scatter(S.om, S.q_or)
    C = oamr.criterion_speed(qL) if criterion == 0 else oamr.criterion_vorticity(S.om, qL)
    cmax = np.sort(C.reshape(S.om.n_elem, -1).max(axis=1))
    lvl = S.om.e_level
    lvl_max = int(lvl.max()) + 1
    # thresholds half-way across gaps between element maxima that are wide
    # compared with round-off (symmetric elements have maxima equal up to a
    # few ulps, and a cut between those would test rounding, not the rule)
    scale = np.abs(cmax).max()
    gaps = np.nonzero(np.diff(cmax) > 1e-8 * scale)[0]
    picks = np.linspace(0.2, 0.8, lvl_max)
    sel = gaps[np.clip((picks * (len(gaps) - 1)).astype(int), 0, len(gaps) - 1)]
    thr = np.sort(0.5 * (cmax[sel] + cmax[sel + 1]))
    ef = oamr.element_flags(C.reshape(S.om.n_elem, -1), lvl, thr, lvl_max)
    cf = oamr.column_flags(ef, S.c["columns"], S.om.n_z)
    ae = torch.zeros(S.gm.info["n_elem"], dtype=torch.int8, device="cuda")
    ac = torch.zeros(S.gm.info["n_col"], dtype=torch.int8, device="cuda")
    api.amr_flag(S.gm, S.q_g, criterion, thr, lvl_max, ae, ac)
    torch.cuda.synchronize()
    assert np.array_equal(ae.cpu().numpy(), ef)
    assert np.array_equal(ac.cpu().numpy(), cf)
    assert len(set(ef.tolist())) >= 2


def test_api_rejects_bad_calls():
    S = get(*CASES[0])
    torch, api = S.torch, S.api
    from paper_2410_21607_amd.native import SemError
    say("bad calls")
    q = S.q_g
    with pytest.raises(SemError):
        api.sem_stage(S.gm, 0.0, 1.0, 1.0, q, q, q, api.SEM_FP64)   # aliasing
    with pytest.raises(SemError):
        api.sem_stage(S.gm, 0.0, 1.0, 1.0, q, q.clone(), torch.zeros_like(q), 7)
    with pytest.raises(SemError):
        api.amr_flag(S.gm, q, 0, [2.0, 1.0], 2,
                     torch.zeros(S.gm.info["n_elem"], dtype=torch.int8, device="cuda"),
                     torch.zeros(S.gm.info["n_col"], dtype=torch.int8, device="cuda"))
    with pytest.raises(ValueError):
        api.sem_stage(S.gm, 0.0, 1.0, 1.0, q[:-1], q.clone(), torch.zeros_like(q))


# work layouts of the fused stage: single columns in chunks of 1, 2, 4, 8
# layers in each FP64 thread order (0: planes between elements first, 2:
# vertical index fastest, 3: split element, two or more layers); 2 x 2 column
# blocks in 1, 2 or 4 vertical segments
TUNES = [(0, 1), (0, 2), (0, 4), (0, 8), (2, 1), (2, 2), (2, 4), (2, 8), (3, 2), (3, 4), (3, 8),
         (1, 1), (1, 2), (1, 4)]
TUNE_IDS = ["col1", "col2", "col4", "col8", "kz1", "kz2", "kz4", "kz8", "split2", "split4", "split8",
            "blk1", "blk2", "blk4"]
DECOMP = [0, 1, 2, 4, 5, 6, 7]


@pytest.mark.parametrize("name,kw", [CASES[k] for k in DECOMP], ids=[IDS[k] for k in DECOMP])
@pytest.mark.parametrize("layout", TUNES, ids=TUNE_IDS)
def test_fused_stage_decompositions(name, kw, layout):
    """Every work layout of the fused stage gives the oracle's stage."""
    S = get(name, kw)
    torch, api = S.torch, S.api
    from paper_2410_21607_amd.native import SemError
    say("fused layout", name, kw, layout)
    saved = api.sem_stage_get_layout(S.gm)
    try:
        api.sem_stage_set_layout(S.gm, *layout)
    except SemError:
        pytest.skip("no kernel instance for this order and layout")
    try:
        assert api.sem_stage_get_layout(S.gm)[0] == layout[0]
        dt = S.c["dt"]
        qn = S.q_g.clone()
        qs = S.q_g.clone()
        out = torch.zeros_like(qn)
        for st in range(3):
            a, b, cc = timestep.stage_coefficients(st, dt)
            api.sem_stage(S.gm, a, b, cc, qn, qs, out, api.SEM_FP64)
            qs, out = out, qs
        torch.cuda.synchronize()
    finally:
        api.sem_stage_set_layout(S.gm, *saved)
    rhs = lambda q: assembly.rhs(S.om, q, S.ref, S.c["phys"])
    want, _ = timestep.run_stages(rhs, S.q_or, dt, 3)
    err = metrics.rel_l2(S.to_oracle_order(qs), want, metrics.STATE_FLOORS)
    say("  rel", err)
    assert err.max() <= TOL64


def test_layouts_agree_with_each_other():
    """The block and column layouts sum the same contributions in different
    orders: on every mesh with blocks their stages agree to 1e-14."""
    for k in DECOMP:
        S = get(*CASES[k])
        torch, api = S.torch, S.api
        if not (3 <= S.c["N"] <= 5):
            continue
        saved = api.sem_stage_get_layout(S.gm)
        outs = []
        try:
            for lay in ((0, 0), (1, 0)):
                api.sem_stage_set_layout(S.gm, *lay)
                out = torch.zeros_like(S.q_g)
                api.sem_stage(S.gm, 0.75, 0.25, 0.25 * S.c["dt"], S.q_g, S.q_g, out, api.SEM_FP64)
                torch.cuda.synchronize()
                outs.append(S.gm.pack(out))
        finally:
            api.sem_stage_set_layout(S.gm, *saved)
        err = metrics.rel_l2(outs[1], outs[0], metrics.STATE_FLOORS)
        say("  layouts", IDS[k], err)
        assert err.max() <= 1e-14


def test_thread_orders_bit_identical():
    """The FP64 thread orders of the column layout assign the same arithmetic
    to every node (each element's part rounded on its own, summed lower
    element first) and sum the columns in the same colour order: a stage (and
    its right-hand side alone) is bit-identical between them, at every chunk
    depth, on every mesh (hanging points and side columns included)."""
    for k in DECOMP:
        S = get(*CASES[k])
        torch, api = S.torch, S.api
        from paper_2410_21607_amd.native import SemError
        saved = api.sem_stage_get_layout(S.gm)
        n_z = S.c["z_edges"].size - 1
        tried = 0
        try:
            for lpc in (1, 2, 4, 8):
                if lpc > 2 * n_z:
                    continue
                outs = []
                for lay in (api.SEM_LAYOUT_COLUMNS, api.SEM_LAYOUT_COLUMNS_KZ,
                            api.SEM_LAYOUT_COLUMNS_SPLIT):
                    try:
                        api.sem_stage_set_layout(S.gm, lay, lpc)
                    except SemError:
                        continue
                    for a, b, cc in ((0.75, 0.25, 0.25 * S.c["dt"]), (0.0, 0.0, 1.0)):
                        out = torch.zeros_like(S.q_g)
                        api.sem_stage(S.gm, a, b, cc, S.q_g, S.q_g, out, api.SEM_FP64)
                        outs.append(out)
                torch.cuda.synchronize()
                if len(outs) < 4:
                    continue
                say("  orders", IDS[k], "lpc", lpc, "layouts compared", len(outs) // 2)
                for j in range(2, len(outs), 2):
                    assert torch.equal(outs[0], outs[j]) and torch.equal(outs[1], outs[j + 1])
                tried += 1
        finally:
            api.sem_stage_set_layout(S.gm, *saved)
        assert tried >= 1


def test_fused_fp32_stage_error():
    """FP32 element arithmetic inside the fused stage, FP64 accumulation."""
    S = get(*CASES[0])
    torch, api = S.torch, S.api
    say("fused fp32")
    dt = S.c["dt"]
    qn = S.q_g.clone()
    qs = S.q_g.clone()
    out = torch.zeros_like(qn)
    for st in range(3):
        a, b, cc = timestep.stage_coefficients(st, dt)
        api.sem_stage(S.gm, a, b, cc, qn, qs, out, api.SEM_FP32)
        qs, out = out, qs
    torch.cuda.synchronize()
    rhs = lambda q: assembly.rhs(S.om, q, S.ref, S.c["phys"])
    want, _ = timestep.run_stages(rhs, S.q_or, dt, 3)
    err = metrics.rel_l2(S.to_oracle_order(qs), want, metrics.STATE_FLOORS)
    say("  rel fp32", err)
    assert err.max() <= 1e-6
