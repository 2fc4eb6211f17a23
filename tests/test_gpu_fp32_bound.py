"""Reduced-precision variant against the oracle's own float32 mode: the GPU
FP32 error (element arithmetic in float32, assembly and update in FP64)
relative to the FP64 oracle must stay within twice the error of the oracle
evaluating the same steps in float32, field by field, for one right-hand side
and after three stages.  Both round p' once from its FP64 value and then take
the same float32 steps, so the two errors differ only by the order of the
roundings in the sums (observed ratio 0.85-1.04)."""

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


@pytest.mark.parametrize("name,kw", [("vortex_8x8x4_n4", {}), ("small_amr3", {}),
                                     ("small_amr2", {"N": 7})])
def test_fp32_within_twice_oracle_fp32(name, kw):
    import torch
    from paper_2410_21607_amd import api
    c = cases.get(name, **kw)
    say("fp32 bound", name, kw)
    gm = api.Mesh.from_case(c)
    _, _, z = gm.coords()
    bg = cases.reference_state(c, z)
    gm.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    om = oracle_mesh(c)
    perm = match(om.node_xyz, gm.node_xyz(), c)
    q = cases.initial_state(c, om.node_xyz)
    ref = oracle_reference_local(c, om)
    f64 = lambda s: assembly.rhs(om, s, ref, c["phys"])
    f32 = lambda s: assembly.rhs(om, s, ref, c["phys"], dtype=np.float32)
    # one right-hand side: the fused stage with (a, b, c) = (0, 0, 1) returns R
    qg = gm.unpack(q[:, perm])
    out = torch.zeros_like(qg)
    api.sem_stage(gm, 0.0, 0.0, 1.0, qg, qg, out, api.SEM_FP32)
    torch.cuda.synchronize()
    got = np.empty_like(q)
    got[:, perm] = gm.pack(out)
    want, ref32 = f64(q), f32(q)
    e_gpu = metrics.rel_l2(got, want, metrics.RHS_FLOORS)
    e_or = metrics.rel_l2(ref32, want, metrics.RHS_FLOORS)
    say("  rhs  gpu", e_gpu, "oracle fp32", e_or)
    assert np.all(e_gpu <= 2.0 * e_or + 1e-13)
    # three stages
    w64, _ = timestep.run_stages(f64, q, c["dt"], 3)
    w32, _ = timestep.run_stages(f32, q, c["dt"], 3)
    qs, o = qg.clone(), torch.zeros_like(qg)
    for s in range(3):
        a, b, cc = timestep.stage_coefficients(s, c["dt"])
        api.sem_stage(gm, a, b, cc, qg, qs, o, api.SEM_FP32)
        qs, o = o, qs
    torch.cuda.synchronize()
    got = np.empty_like(q)
    got[:, perm] = gm.pack(qs)
    e_gpu = metrics.rel_l2(got, w64, metrics.STATE_FLOORS)
    e_or = metrics.rel_l2(w32, w64, metrics.STATE_FLOORS)
    say("  3 stages gpu", e_gpu, "oracle fp32", e_or)
    assert np.all(e_gpu <= 2.0 * e_or + 1e-15)
