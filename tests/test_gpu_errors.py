"""Error paths of the device entry points added for adaptation, the
forecaster and the dissipation: every bad call returns an error code (raised
as SemError by the binding) before launching anything."""

import numpy as np
import pytest

from synth import cases

pytestmark = pytest.mark.gpu


def test_device_entry_points_reject_bad_calls():
    import torch
    from paper_2410_21607_amd import api, native
    c = cases.get("small_amr3", N=3)
    gm = api.Mesh.from_case(c)
    other = api.Mesh.from_case(cases.get("small_amr3", N=4))
    with pytest.raises(native.SemError):
        api.Transfer(gm, other)                       # different orders
    T = api.Transfer(gm, gm)
    q = gm.state()
    with pytest.raises(native.SemError):
        native.call("sem_transfer_apply", T.handle, api._ptr(q, torch.float64, gm.n_state, "q"),
                    api._ptr(q, torch.float64, gm.n_state, "q"), None)   # aliasing
    ne = gm.info["n_elem"]
    feat = torch.zeros(ne * 16, dtype=torch.float32, device="cuda")
    dem = torch.zeros(ne, dtype=torch.int8, device="cuda")
    plain = torch.zeros(ne, dtype=torch.int8, device="cuda")
    with pytest.raises(native.SemError):              # reference state not set yet
        api.amr_features(gm, q, q, plain, 1, [1e-4], 1, np.ones(16), feat, dem)
    _, _, z = gm.coords()
    bg = cases.reference_state(c, z)
    gm.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    with pytest.raises(native.SemError):              # decreasing thresholds
        api.amr_features(gm, q, q, plain, 1, [2e-4, 1e-4], 2, np.ones(16), feat, dem)
    with pytest.raises(native.SemError):
        gm.set_dissipation(-1.0, 0.0, 1.0)
    with pytest.raises(native.SemError):
        gm.set_dissipation(0.0, 1.0, 0.0)             # a layer needs a depth
    P = torch.zeros(api.MLP_NPARAM, dtype=torch.float32, device="cuda")
    with pytest.raises(native.SemError):
        api.mlp_adam_step(P, P, P.clone(), P.clone(), 0)   # step count starts at 1
    x = torch.zeros(4 * 16, dtype=torch.float32, device="cuda").view(4, 16)
    y = torch.zeros(4, dtype=torch.int8, device="cuda")
    idx = torch.zeros(0, dtype=torch.int32, device="cuda")
    with pytest.raises(native.SemError):              # empty batch
        api.mlp_backward(P, x, y, idx, torch.zeros(1, device="cuda"), P.clone(),
                         torch.zeros(1, device="cuda"))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(native.SemError):              # empty box
        api.sem_max_wind(gm, q, (1.0, 0.0, 0.0, 1.0), out)
    torch.cuda.synchronize()
