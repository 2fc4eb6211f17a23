"""GPU parity of the terrain-following fused stage (sem_stage after
sem_mesh_set_terrain) against the oracle's mapped elements (oracle.terrain):

* the right-hand side itself (a stage with a = b = 0, c = 1), on hills and on
  a plane slope, uniform and 2:1 nonconforming meshes, N = 3 to 7, every
  supported chunk depth;
* several SSP-RK3 stages;
* the unfused calls (scatter, sem_rhs, assemble, gather, finalize) against
  the oracle and against the fused stage;
* flat terrain against the box-element stage;
* the refinement flags over terrain (both criteria, bit-exact) and the
  forecaster features (with the criterion's level, bit-exact);
* SEM_FP32 over terrain against the oracle's float32 mapped elements;
* the horizontal Smagorinsky-Lilly and absorbing-layer terms over terrain;
* the error paths (heights out of range, non-positive reference).

Bar: floor-scaled relative L2 <= 1e-12 per field (FP64); SEM_FP32 within twice
the oracle's own float32 error per field."""

import sys

import numpy as np
import pytest

from harness import match, oracle_mesh
from oracle import amr as oamr
from oracle import assembly, metrics, timestep
from oracle import terrain as oterrain
from synth import cases

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def hills(c, amp=1500.0):
    kx, ky = 2 * np.pi / c["Lx"], 2 * np.pi / c["Ly"]
    return lambda x, y: 0.5 * amp * (1.0 + np.cos(kx * x) * np.cos(ky * y + 0.4))


def slope(c, s=0.004):
    return lambda x, y: s * (x + 0.5 * c["Lx"]) + 0.001 * (y + 0.5 * c["Ly"])


class Setup:
    def __init__(self, name, kw, shape, periodic=True):
        import torch
        from paper_2410_21607_amd import api
        self.torch, self.api = torch, api
        c = cases.get(name, **dict(kw))
        c["periodic_x"] = c["periodic_y"] = periodic
        self.c = c
        self.om = oracle_mesh(c)
        self.gm = api.Mesh.from_case(c)
        self.perm = match(self.om.node_xyz, self.gm.node_xyz(), c)
        fn = hills(c) if shape == "hills" else slope(c)
        self.zs = fn(self.om.node_xyz[:, 0], self.om.node_xyz[:, 1])
        zp = oterrain.node_heights(self.om, self.zs)
        bg = cases.reference_state(c, zp)
        self.ref = dict(rho0=bg["rho0"], theta0=bg["theta0"], dtheta0dz=bg["dtheta0dz"])
        xyz = self.om.node_xyz.copy()
        xyz[:, 2] = zp
        self.q_or = cases.initial_state(c, xyz)
        nzn = self.gm.info["nzn"]
        zs_nodes = self.zs[self.perm].reshape(-1, nzn)
        assert np.all(zs_nodes == zs_nodes[:, :1])      # constant along every column
        self.gm.set_terrain(zs_nodes[:, 0], *(self.ref[k][self.perm]
                                             for k in ("rho0", "theta0", "dtheta0dz")))
        # the library's physical heights agree with the oracle's, both under
        # the surface passed in and under the one now set on the handle
        np.testing.assert_allclose(self.gm.heights(), zp[self.perm], rtol=0, atol=1e-9)
        np.testing.assert_allclose(self.gm.heights(zs_nodes[:, 0]), zp[self.perm], rtol=0, atol=1e-9)
        self.q_g = self.gm.unpack(self.q_or[:, self.perm])

    def to_oracle_order(self, flat):
        a = self.gm.pack(flat)
        out = np.empty_like(a)
        out[:, self.perm] = a
        return out

    def oracle_rhs(self, q):
        return oterrain.rhs(self.om, q, self.ref, self.zs, self.c["phys"])

    def gpu_rhs(self):
        out = self.torch.zeros_like(self.q_g)
        self.api.sem_stage(self.gm, 0.0, 0.0, 1.0, self.q_g, self.q_g.clone(), out)
        self.torch.cuda.synchronize()
        return self.to_oracle_order(out)


CASES = [("vortex_8x8x4_n4", {}, "hills", True),
         ("small_amr2", {}, "hills", True),
         ("small_amr3", {"N": 5}, "slope", False),
         ("small_uniform", {"N": 3}, "hills", True),
         ("small_uniform", {"N": 7}, "slope", False),
         ("vortex_8x8x4_n4", {"N": 5}, "slope", False),
         ("small_uniform", {"N": 6}, "hills", False),
         ("small_amr2", {"N": 7}, "hills", True),
         ("small_amr3", {"N": 3}, "hills", True)]
IDS = [f"{n}-{kw}-{s}-{'per' if p else 'wall'}" for n, kw, s, p in CASES]


@pytest.mark.parametrize("name,kw,shape,periodic", CASES, ids=IDS)
def test_terrain_rhs_matches_oracle_every_chunk_depth(name, kw, shape, periodic):
    S = Setup(name, kw, shape, periodic)
    want = S.oracle_rhs(S.q_or)
    n_z = S.c["z_edges"].size - 1
    tried = 0
    for lpc in (1, 2, 4, 8):
        if lpc > 2 * n_z:
            continue
        try:
            S.api.sem_stage_tune(S.gm, lpc)
        except Exception:
            continue                               # no instance at this order
        say("terrain rhs", name, kw, shape, "lpc", lpc)
        got = S.gpu_rhs()
        err = metrics.rel_l2(got, want, metrics.RHS_FLOORS)
        say("  rel", err)
        assert err.max() <= TOL64
        # the other FP64 thread orders: the same values, bit for bit
        S.api.sem_stage_set_layout(S.gm, S.api.SEM_LAYOUT_COLUMNS_KZ, lpc)
        assert np.array_equal(S.gpu_rhs(), got)
        if lpc > 1:
            try:
                S.api.sem_stage_set_layout(S.gm, S.api.SEM_LAYOUT_COLUMNS_SPLIT, lpc)
            except Exception:
                pass                               # a pair across two waves
            else:
                assert np.array_equal(S.gpu_rhs(), got)
        tried += 1
    assert tried >= 2


@pytest.mark.parametrize("name,kw,shape,periodic", CASES[:4] + CASES[7:], ids=IDS[:4] + IDS[7:])
def test_terrain_unfused_calls_match_oracle_and_fused_stage(name, kw, shape, periodic):
    """sem_nc_project(SCATTER) -> sem_rhs -> sem_dss(ASSEMBLE) ->
    sem_nc_project(GATHER) -> sem_dss(FINALIZE) over terrain."""
    S = Setup(name, kw, shape, periodic)
    torch, api = S.torch, S.api
    say("terrain unfused", name, kw, shape)
    n, nh, nl = S.gm.n_state, S.gm.n_hstate, 5 * S.gm.n_local
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda")
    hv, rE, acc, cH, r = z(nh), z(nl), z(n), z(nh), z(n)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_SCATTER, S.q_g, hv)
    api.sem_rhs(S.gm, S.q_g, hv if nh else None, rE)
    api.sem_dss(S.gm, api.SEM_ASSEMBLE, rE=rE, acc=acc, c=cH if nh else None)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_GATHER, cH, acc)
    api.sem_dss(S.gm, api.SEM_FINALIZE, acc=acc, r=r)
    torch.cuda.synchronize()
    got = S.to_oracle_order(r)
    err = metrics.rel_l2(got, S.oracle_rhs(S.q_or), metrics.RHS_FLOORS)
    say("  rel vs oracle", err)
    assert err.max() <= TOL64
    fused = S.gpu_rhs()
    errf = metrics.rel_l2(got, fused, metrics.RHS_FLOORS)
    say("  rel vs fused", errf)
    assert errf.max() <= 1e-13


@pytest.mark.parametrize("name,kw,shape,periodic", CASES[:3], ids=IDS[:3])
def test_terrain_stages_match_oracle(name, kw, shape, periodic):
    S = Setup(name, kw, shape, periodic)
    torch, api = S.torch, S.api
    nst, dt = 6, S.c["dt"]
    say("terrain stages", name, kw, shape, nst)
    qn, qs = S.q_g.clone(), S.q_g.clone()
    out = torch.zeros_like(qn)
    for st in range(nst):
        a, b, cc = timestep.stage_coefficients(st % 3, dt)
        api.sem_stage(S.gm, a, b, cc, qn, qs, out)
        qs, out = out, qs
        if st % 3 == 2:
            qn.copy_(qs)
    torch.cuda.synchronize()
    want, _ = timestep.run_stages(S.oracle_rhs, S.q_or, dt, nst)
    err = metrics.rel_l2(S.to_oracle_order(qs), want, metrics.STATE_FLOORS)
    say("  rel", err)
    assert err.max() <= TOL64


@pytest.mark.parametrize("name,kw,shape,periodic", [CASES[0], CASES[1], CASES[2], CASES[4]],
                         ids=[IDS[0], IDS[1], IDS[2], IDS[4]])
@pytest.mark.parametrize("criterion", [0, 1])
def test_terrain_amr_flag_bit_exact(name, kw, shape, periodic, criterion):
    """The refinement flags over terrain: |u| needs no metric; the vorticity
    takes the chain rule of the mapping (oracle: full inverse Jacobian)."""
    S = Setup(name, kw, shape, periodic)
    torch, api = S.torch, S.api
    say("terrain amr_flag", name, kw, shape, criterion)
    qL = assembly.scatter(S.om, S.q_or)
    C = oamr.criterion_speed(qL) if criterion == 0 else oterrain.criterion_vorticity(S.om, qL, S.zs)
    cmax = np.sort(C.reshape(S.om.n_elem, -1).max(axis=1))
    lvl = S.om.e_level
    lvl_max = int(lvl.max()) + 1
    # thresholds half-way across gaps between element maxima that are wide
    # compared with round-off
    gaps = np.nonzero(np.diff(cmax) > 1e-8 * np.abs(cmax).max())[0]
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


def test_flat_terrain_matches_the_box_element_stage():
    import torch
    from paper_2410_21607_amd import api
    c = cases.get("vortex_8x8x4_n4")
    gm = api.Mesh.from_case(c)
    _, _, z = gm.coords()
    bg = cases.reference_state(c, z)
    gm.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    q = gm.unpack(cases.initial_state(c, gm.node_xyz()))
    box = torch.zeros_like(q)
    api.sem_stage(gm, 0.0, 0.0, 1.0, q, q.clone(), box)
    nzn = z.size
    nodes = cases.reference_state(c, np.tile(z, gm.info["n_h"]))
    gm.set_terrain(np.zeros(gm.info["n_h"]), nodes["rho0"], nodes["theta0"], nodes["dtheta0dz"])
    ter = torch.zeros_like(q)
    api.sem_stage(gm, 0.0, 0.0, 1.0, q, q.clone(), ter)
    gm.set_terrain(None)
    again = torch.zeros_like(q)
    api.sem_stage(gm, 0.0, 0.0, 1.0, q, q.clone(), again)
    torch.cuda.synchronize()
    assert torch.equal(again, box)                 # removing the terrain restores the box path
    b, t = gm.pack(box), gm.pack(ter)
    scale = np.abs(b).max(axis=1, keepdims=True)
    assert nzn > 0 and np.all(np.abs(t - b) <= 1e-13 * scale)


def test_terrain_error_paths():
    from paper_2410_21607_amd import api, native
    c = cases.get("small_uniform", N=3)
    gm = api.Mesh.from_case(c)
    nh, n = gm.info["n_h"], gm.n_dof
    one, zero = np.ones(n), np.zeros(n)
    for bad in (np.full(nh, -1.0), np.full(nh, 20e3), np.full(nh, np.nan)):
        with pytest.raises(native.SemError) as e:  # heights outside [0, H - z0)
            gm.set_terrain(bad, one, 300 * one, zero)
        assert e.value.code == -1
    with pytest.raises(native.SemError):           # non-positive reference
        gm.set_terrain(np.zeros(nh), zero, 300 * one, zero)
    gm.set_terrain(np.full(nh, 500.0), one, 300 * one, zero)
    gm.set_dissipation(0.21, 0.0, 4000.0)           # the terms combine with terrain
    gm.set_terrain(None)


FEAT_SCALE = np.array([1.0, 1e3, 1e3, 0.05, 1.0, 1.0, 1.0, 20.0, 1e3, 1e4, 1e3, 1e3, 0.05, 0.5,
                       1e4, 1.0])


@pytest.mark.parametrize("name,kw,shape,periodic", [CASES[0], CASES[1], CASES[2], CASES[7]],
                         ids=[IDS[0], IDS[1], IDS[2], IDS[7]])
@pytest.mark.parametrize("criterion", [0, 1])
def test_terrain_features_match_oracle(name, kw, shape, periodic, criterion):
    """Forecaster features over terrain (physical derivatives by the chain
    rule, p' from the per-node reference) against the oracle's, and the level
    the criterion asks for, bit-exact."""
    from oracle import forecast
    S = Setup(name, kw, shape, periodic)
    torch, api = S.torch, S.api
    say("terrain features", name, kw, shape, criterion)
    rng = np.random.default_rng(5)
    qp = S.q_or * (1.0 + 0.05 * rng.standard_normal(S.q_or.shape))
    qL, qLp = assembly.scatter(S.om, S.q_or), assembly.scatter(S.om, qp)
    refL = {k: assembly.scatter(S.om, S.ref[k][None])[0] for k in ("rho0", "theta0")}
    ne = S.om.n_elem
    C = oamr.criterion_speed(qL) if criterion == 0 else oterrain.criterion_vorticity(S.om, qL, S.zs)
    cmax = np.unique(C.reshape(ne, -1).max(axis=1))
    gaps = np.argsort(np.diff(cmax))[::-1][:2]      # the two widest gaps
    thr = np.sort(0.5 * (cmax[gaps] + cmax[gaps + 1]))
    plain = rng.integers(-1, 2, size=ne).astype(np.int8)
    want, dem_o = forecast.features(S.om, qL, qLp, plain, refL, S.c["phys"], criterion, thr, 2,
                                    FEAT_SCALE, zsG=S.zs)
    feat = torch.zeros(ne * 16, dtype=torch.float32, device="cuda")
    dem = torch.zeros(ne, dtype=torch.int8, device="cuda")
    api.amr_features(S.gm, S.q_g, S.gm.unpack(qp[:, S.perm]), torch.as_tensor(plain).cuda(),
                     criterion, thr, 2, FEAT_SCALE, feat, dem)
    torch.cuda.synchronize()
    got = feat.cpu().numpy().reshape(ne, 16).astype(np.float64)
    say("  worst relative error per feature", (np.abs(got - want) / (np.abs(want) + 1e-3)).max(0))
    assert np.all(np.abs(got - want) <= 2e-6 * np.abs(want) + 1e-6)
    np.testing.assert_array_equal(dem.cpu().numpy(), dem_o)
    assert len(set(dem_o.tolist())) >= 2


@pytest.mark.parametrize("name,kw,shape,periodic", [CASES[0], CASES[1], CASES[2], CASES[7]],
                         ids=[IDS[0], IDS[1], IDS[2], IDS[7]])
def test_terrain_fp32_within_twice_oracle_fp32(name, kw, shape, periodic):
    """SEM_FP32 over terrain (element arithmetic in float32, metric factors
    from FP64, p' rounded once from FP64, assembly and update in FP64): the
    error against the FP64 oracle stays within twice the error of the oracle's
    float32 mapped elements, field by field, for the right-hand side (the fused
    stage at every chunk depth and the unfused calls) and after three stages
    (observed ratio 0.92-1.04)."""
    S = Setup(name, kw, shape, periodic)
    torch, api = S.torch, S.api
    f64 = S.oracle_rhs
    f32 = lambda q: oterrain.rhs(S.om, q, S.ref, S.zs, S.c["phys"], dtype=np.float32)
    want, ref32 = f64(S.q_or), f32(S.q_or)
    e_or = metrics.rel_l2(ref32, want, metrics.RHS_FLOORS)
    say("terrain fp32", name, kw, shape, "oracle fp32", e_or)
    n_z = S.c["z_edges"].size - 1
    tried = 0
    for lpc in (1, 2, 4, 8):
        if lpc > 2 * n_z:
            continue
        try:
            api.sem_stage_tune(S.gm, lpc)
        except Exception:
            continue                               # no instance at this order
        out = torch.zeros_like(S.q_g)
        api.sem_stage(S.gm, 0.0, 0.0, 1.0, S.q_g, S.q_g.clone(), out, api.SEM_FP32)
        torch.cuda.synchronize()
        e_gpu = metrics.rel_l2(S.to_oracle_order(out), want, metrics.RHS_FLOORS)
        say("  fused lpc", lpc, e_gpu)
        assert np.all(e_gpu <= 2.0 * e_or + 1e-13)
        tried += 1
    assert tried >= 2
    # unfused: scatter -> sem_rhs(FP32) -> assemble -> gather -> finalize
    n, nh, nl = S.gm.n_state, S.gm.n_hstate, 5 * S.gm.n_local
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda")
    hv, rE, acc, cH, r = z(nh), z(nl), z(n), z(nh), z(n)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_SCATTER, S.q_g, hv)
    api.sem_rhs(S.gm, S.q_g, hv if nh else None, rE, api.SEM_FP32)
    api.sem_dss(S.gm, api.SEM_ASSEMBLE, rE=rE, acc=acc, c=cH if nh else None)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_GATHER, cH, acc)
    api.sem_dss(S.gm, api.SEM_FINALIZE, acc=acc, r=r)
    torch.cuda.synchronize()
    e_gpu = metrics.rel_l2(S.to_oracle_order(r), want, metrics.RHS_FLOORS)
    say("  unfused", e_gpu)
    assert np.all(e_gpu <= 2.0 * e_or + 1e-13)
    # three stages (the autotuner's pick of the chunk depth)
    q0 = S.q_g.clone()
    lpc, ms = api.sem_stage_autotune(S.gm, q0, q0.clone(), torch.zeros_like(q0), api.SEM_FP32)
    say("  autotune fp32", lpc, ms)
    assert lpc >= 1 and ms > 0.0
    dt = S.c["dt"]
    w64, _ = timestep.run_stages(f64, S.q_or, dt, 3)
    w32, _ = timestep.run_stages(f32, S.q_or, dt, 3)
    qs, o = S.q_g.clone(), torch.zeros_like(S.q_g)
    for st in range(3):
        a, b, cc = timestep.stage_coefficients(st, dt)
        api.sem_stage(S.gm, a, b, cc, S.q_g, qs, o, api.SEM_FP32)
        qs, o = o, qs
    torch.cuda.synchronize()
    e_gpu = metrics.rel_l2(S.to_oracle_order(qs), w64, metrics.STATE_FLOORS)
    e_or3 = metrics.rel_l2(w32, w64, metrics.STATE_FLOORS)
    say("  3 stages gpu", e_gpu, "oracle fp32", e_or3)
    assert np.all(e_gpu <= 2.0 * e_or3 + 1e-15)


def _unfused_rhs(S, precision=None):
    """scatter -> sem_rhs -> assemble -> gather -> finalize, in oracle order."""
    torch, api = S.torch, S.api
    n, nh, nl = S.gm.n_state, S.gm.n_hstate, 5 * S.gm.n_local
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda")
    hv, rE, acc, cH, r = z(nh), z(nl), z(n), z(nh), z(n)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_SCATTER, S.q_g, hv)
    api.sem_rhs(S.gm, S.q_g, hv if nh else None, rE,
                api.SEM_FP64 if precision is None else precision)
    api.sem_dss(S.gm, api.SEM_ASSEMBLE, rE=rE, acc=acc, c=cH if nh else None)
    if nh:
        api.sem_nc_project(S.gm, api.SEM_GATHER, cH, acc)
    api.sem_dss(S.gm, api.SEM_FINALIZE, acc=acc, r=r)
    torch.cuda.synchronize()
    return S.to_oracle_order(r)


@pytest.mark.parametrize("name,kw,shape,periodic", [CASES[0], CASES[1], CASES[2], CASES[7]],
                         ids=[IDS[0], IDS[1], IDS[2], IDS[7]])
def test_terrain_dissipation_matches_oracle(name, kw, shape, periodic):
    """Horizontal Smagorinsky-Lilly and the absorbing layer over terrain
    (physical derivatives, layer at the physical height) against the oracle's
    mapped-element terms: the unfused calls, the fused stage (right-hand side
    and three stages), the dissipation part on its own scale, and switching
    the terms off again."""
    S = Setup(name, kw, shape, periodic)
    torch, api = S.torch, S.api
    say("terrain dissipation", name, kw, shape)
    phys = dict(S.c["phys"], Cs=0.21, sponge_gamma=0.05, sponge_depth=8000.0)
    r_off = _unfused_rhs(S)
    S.gm.set_dissipation(0.21, 0.05, 8000.0)
    r_on = _unfused_rhs(S)
    want_on = oterrain.rhs(S.om, S.q_or, S.ref, S.zs, phys)
    want_off = S.oracle_rhs(S.q_or)
    err = metrics.rel_l2(r_on, want_on, metrics.RHS_FLOORS)
    dd = want_on - want_off
    floors = np.maximum(np.abs(dd).max(axis=1), 1e-300) * 1e-3
    err_d = metrics.rel_l2(r_on - r_off, dd, floors)
    say("  unfused rel", err, "dissipation part rel", err_d)
    assert np.abs(dd[1]).max() > 0 and np.abs(dd[0]).max() > 0
    assert err.max() <= TOL64 and err_d.max() <= 1e-9
    fused = S.gpu_rhs()
    errf = metrics.rel_l2(fused, want_on, metrics.RHS_FLOORS)
    say("  fused rel", errf)
    assert errf.max() <= TOL64
    dt = S.c["dt"]
    want, _ = timestep.run_stages(lambda q: oterrain.rhs(S.om, q, S.ref, S.zs, phys), S.q_or, dt, 3)
    qs, o = S.q_g.clone(), torch.zeros_like(S.q_g)
    for st in range(3):
        a, b, cc = timestep.stage_coefficients(st, dt)
        api.sem_stage(S.gm, a, b, cc, S.q_g, qs, o)
        qs, o = o, qs
    torch.cuda.synchronize()
    err3 = metrics.rel_l2(S.to_oracle_order(qs), want, metrics.STATE_FLOORS)
    say("  3 stages rel", err3)
    assert err3.max() <= TOL64
    S.gm.set_dissipation(0.0, 0.0, 8000.0)
    assert np.array_equal(_unfused_rhs(S), r_off)


def _mountain_hook(case, amp=1000.0, half_width=40e3):
    """Terrain hook of an adaptive run: a Gaussian mountain, reference state
    per node at the nodes' physical heights."""

    def hook(mesh):
        hxy, _, zf = mesh.coords()
        zs = amp * np.exp(-(hxy[:, 0] ** 2 + hxy[:, 1] ** 2) / half_width ** 2)
        bg = cases.reference_state(case, mesh.heights(zs))
        return zs, bg["rho0"], bg["theta0"], bg["dtheta0dz"]
    return hook


@pytest.mark.timeout(300)
def test_adaptive_run_over_terrain_matches_uniform_finest():
    """Criterion-driven adaptation (split, balance, merge, transfer) over a
    mountain keeps the maximum wind within 1 % of the uniform finest mesh over
    the same mountain, with fewer nodes."""
    import torch
    from paper_2410_21607_amd import api
    from paper_2410_21607_amd.adaptive import AdaptiveRun
    from synth import columns as sc
    c = cases.get("small_vortex3")
    c["amr"] = dict(c["amr"], interval=50)
    c["steer"] = (25.0, 0.0)
    hook = _mountain_hook(c)
    a = c["amr"]
    n_steps = 6 * a["interval"]

    def run(cols, adapt):
        cc = dict(c, columns=cols)
        mesh = api.Mesh.from_case(cc)
        _, _, z = mesh.coords()
        bg = cases.reference_state(cc, z)
        ref = (bg["rho0"], bg["theta0"], bg["dtheta0dz"])
        mesh.set_reference(*ref)
        mesh.set_terrain(*hook(mesh))
        xyz = mesh.node_xyz()
        xyz[:, 2] = mesh.heights()
        q0 = mesh.unpack(cases.initial_state(cc, xyz))
        r = AdaptiveRun(mesh, q0, cc["dt"], ref, a["criterion"], a["thresholds"], a["lvl_max"],
                        a["interval"], adapt=adapt, terrain=hook)
        r.run(n_steps)
        torch.cuda.synchronize()
        return r
    lm = a["lvl_max"]
    fine = np.array([(lm, x, y) for x in range(c["nx0"] << lm) for y in range(c["ny0"] << lm)])
    say("adaptive over terrain: uniform finest")
    uni = run(sc.morton_sort(fine, lm), False)
    say("adaptive over terrain: adaptive")
    amr = run(np.asarray(c["columns"]), True)
    vu = np.array([b["vmax"] for b in uni.log])
    va = np.array([b["vmax"] for b in amr.log])
    dev = np.max(np.abs(va - vu) / vu)
    say("  rebuilds", amr.n_rebuild, "max-wind deviation", dev,
        "mean nodes", np.mean([b["n_dof"] for b in amr.log]), "vs", uni.mesh.n_dof)
    assert np.all(np.isfinite(va)) and np.all(np.isfinite(vu))
    assert amr.n_rebuild >= 1
    assert dev <= 0.01
    assert np.mean([b["n_dof"] for b in amr.log]) < 0.5 * uni.mesh.n_dof
