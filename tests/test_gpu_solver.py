"""GPU tests of the time-stepping layer: the SSP-RK3 stepper against the
oracle, HIP-graph replays against eager execution (every replay checked,
with eager work and synchronisations between replays), determinism, and the
autotuner."""

import sys

import numpy as np
import pytest

from harness import match, oracle_mesh, oracle_reference_local
from oracle import assembly, metrics, timestep
from synth import cases

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup(name, **kw):
    import torch
    from paper_2410_21607_amd import api
    c = cases.get(name, **kw)
    gm = api.Mesh.from_case(c)
    _, _, z = gm.coords()
    bg = cases.reference_state(c, z)
    gm.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    om = oracle_mesh(c)
    perm = match(om.node_xyz, gm.node_xyz(), c)
    q_or = cases.initial_state(c, om.node_xyz)
    q_g = gm.unpack(q_or[:, perm])
    return c, gm, om, perm, q_or, q_g


def to_oracle(flat, perm, gm):
    a = gm.pack(flat)
    out = np.empty_like(a)
    out[:, perm] = a
    return out


@pytest.mark.parametrize("name,kw", [("vortex_8x8x4_n4", {}), ("small_amr3", {"N": 5})])
def test_stepper_matches_oracle(name, kw):
    from paper_2410_21607_amd.solver import Stepper
    c, gm, om, perm, q_or, q_g = setup(name, **kw)
    say("stepper", name, kw)
    st = Stepper(gm, q_g, c["dt"])
    st.step(2)
    import torch
    torch.cuda.synchronize()
    ref = oracle_reference_local(c, om)
    want, _ = timestep.run_stages(lambda q: assembly.rhs(om, q, ref, c["phys"]), q_or, c["dt"], 6)
    err = metrics.rel_l2(to_oracle(st.q, perm, gm), want, metrics.STATE_FLOORS)
    say("  rel", err)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("name,kw", [("vortex_8x8x4_n4", {}), ("small_amr2", {"N": 7})])
def test_graph_replays_equal_eager(name, kw):
    import torch
    from paper_2410_21607_amd.solver import Stepper
    c, gm, om, perm, q_or, q_g = setup(name, **kw)
    say("graph", name, kw)
    eager = Stepper(gm, q_g, c["dt"])
    graph = Stepper(gm, q_g, c["dt"], graph=True)
    for k in range(4):
        graph.step()
        torch.cuda.synchronize()
        eager.step()
        torch.cuda.synchronize()
        # the fused stage is deterministic: replays must match bit for bit
        assert torch.equal(graph.q, eager.q), f"replay {k} differs"
        _ = (eager.q * 2.0).sum().item()      # unrelated eager work between replays


def test_fused_stage_is_deterministic():
    import torch
    from paper_2410_21607_amd import api
    c, gm, om, perm, q_or, q_g = setup("small_amr3", N=7)
    say("determinism")
    outs = []
    for _ in range(3):
        o = torch.zeros_like(q_g)
        api.sem_stage(gm, 0.75, 0.25, 0.1, q_g, q_g, o, api.SEM_FP64)
        torch.cuda.synchronize()
        outs.append(o)
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[1], outs[2])


def test_autotune_then_parity():
    import torch
    from paper_2410_21607_amd import api
    c, gm, om, perm, q_or, q_g = setup("vortex_8x8x4_n4")
    say("autotune")
    scratch = torch.zeros_like(q_g)
    lpc, ms = api.sem_stage_autotune(gm, q_g, q_g.clone(), scratch, api.SEM_FP64, reps=3)
    say("  chosen layers_per_chunk", lpc, "ms", ms)
    assert lpc in (1, 2, 4, 8) and ms > 0
    assert api.sem_stage_get_tune(gm) == lpc
    say("  layout", api.sem_stage_get_layout(gm))
    out = torch.zeros_like(q_g)
    a, b, cc = timestep.stage_coefficients(0, c["dt"])
    api.sem_stage(gm, a, b, cc, q_g, q_g, out, api.SEM_FP64)
    torch.cuda.synchronize()
    ref = oracle_reference_local(c, om)
    want, _ = timestep.run_stages(lambda q: assembly.rhs(om, q, ref, c["phys"]), q_or, c["dt"], 1)
    err = metrics.rel_l2(to_oracle(out, perm, gm), want, metrics.STATE_FLOORS)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_hydrostatic_rest_stays_at_rest(precision):
    """1002 stages (334 RK3 steps, HIP graphs) from the hydrostatic reference
    state with zero perturbation: the wind stays below 1e-10 m/s."""
    import torch
    from paper_2410_21607_amd.solver import Stepper
    c, gm, om, perm, q_or, q_g = setup("small_amr3")
    say("rest", precision)
    st = Stepper(gm, torch.zeros_like(q_g), c["dt"], precision, graph=True)
    st.step(334)
    torch.cuda.synchronize()
    q = gm.pack(st.q)
    assert np.all(np.isfinite(q))
    assert np.abs(q[1:4]).max() <= 1e-10


def test_graph_recaptured_after_mesh_changes():
    """A captured RK3 step holds the fused tables of its capture.  Re-tuning
    (which frees and rebuilds them), or switching the dissipation on and off,
    bumps the mesh's set-up epoch; the stepper must capture again before its
    next replay, and the replays must still match eager steps bit for bit."""
    import torch
    from paper_2410_21607_amd import api
    from paper_2410_21607_amd.solver import Stepper
    c, gm, om, perm, q_or, q_g = setup("small_amr2")
    say("graph epoch")
    eager = Stepper(gm, q_g, c["dt"])
    graph = Stepper(gm, q_g, c["dt"], graph=True)
    assert graph.captures == 1
    e0 = gm.epoch()
    graph.step()
    eager.step()
    torch.cuda.synchronize()
    assert torch.equal(graph.q, eager.q)
    for k, change in enumerate((lambda: api.sem_stage_tune(gm, 1),
                                lambda: api.sem_stage_set_layout(gm, api.SEM_LAYOUT_BLOCKS, 2),
                                lambda: gm.set_dissipation(0.0, 0.0))):
        change()
        assert gm.epoch() > e0
        e0 = gm.epoch()
        graph.step()
        eager.step()
        torch.cuda.synchronize()
        assert graph.captures == 2 + k, "stale graph replayed"
        assert torch.equal(graph.q, eager.q), f"replay after change {k} differs"
    # no change, no capture
    graph.step()
    eager.step()
    torch.cuda.synchronize()
    assert graph.captures == 4 and torch.equal(graph.q, eager.q)
    api.sem_stage_set_layout(gm, api.SEM_LAYOUT_COLUMNS, 0)
