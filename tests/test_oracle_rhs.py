"""Pins of the oracle right-hand side (Section 2), time stepping (Section 5)
and refinement flags (Section 4.1)."""

import itertools

import numpy as np
import pytest

from oracle.mesh import OracleMesh
from oracle import assembly, timestep, amr
from synth import cases, columns, atmosphere


def build(c):
    return OracleMesh(c["N"], c["nx0"], c["ny0"], c["Lx"], c["Ly"], c["z_edges"],
                      c["columns"], c["periodic_x"], c["periodic_y"])


def ref_local(c, m):
    bg = cases.reference_state(c, m.zl)
    return dict(rho0=bg["rho0"], theta0=bg["theta0"], dtheta0dz=bg["dtheta0dz"])


@pytest.mark.parametrize("name,kw", [("vortex_8x8x4_n4", {}), ("small_amr2", {}),
                                     ("small_amr3", {"N": 7})])
@pytest.mark.parametrize("f", [0.0, 5e-5])
def test_constant_free_stream(name, kw, f):
    """rho' = theta' = 0, u = (U, V, 0): R = (0, f V, -f U, 0, 0)."""
    c = cases.get(name, **kw)
    c["phys"]["f"] = f
    m = build(c)
    U, V = 7.0, -3.0
    q = np.zeros((5, m.n_dof))
    q[1], q[2] = U, V
    R = assembly.rhs(m, q, ref_local(c, m), c["phys"])
    expect = np.array([0.0, f * V, -f * U, 0.0, 0.0])
    for k in range(5):
        assert np.abs(R[k] - expect[k]).max() < 1e-16 * 1e3 * max(1.0, abs(U))


@pytest.mark.parametrize("name,kw", [("vortex_8x8x4_n4", {}), ("small_amr3", {"N": 7})])
def test_hydrostatic_rest_is_exactly_steady(name, kw):
    c = cases.get(name, **kw)
    m = build(c)
    R = assembly.rhs(m, np.zeros((5, m.n_dof)), ref_local(c, m), c["phys"])
    assert np.all(R == 0.0)


def test_rk3_amplification_factor():
    """Three stages on dq/dt = lambda q give 1 + z + z^2/2 + z^3/6."""
    for z in (-0.1, -0.5, 0.3 + 0.4j, -1.2):
        lam, dt = z, 1.0
        q = np.array([1.0 + 0j])
        out, _ = timestep.run_stages(lambda s: lam * s, q, dt, 3)
        assert abs(out[0] - (1 + z + z**2 / 2 + z**3 / 6)) < 1e-15


def test_rk3_third_order():
    """Global error of q' = -q + cos t at t=1 falls like dt^3."""
    def solve(n):
        dt = 1.0 / n
        t = [0.0]
        # time-dependent RHS: carry t in the stage driver by hand
        qn = np.array([1.0])
        for _ in range(n):
            qs = qn.copy()
            for s, tau in zip(range(3), (0.0, 1.0, 0.5)):
                a, b, cc = timestep.stage_coefficients(s, dt)
                qs = timestep.stage_update(a, b, cc, qn, qs, -qs + np.cos(t[0] + tau * dt))
            qn = qs
            t[0] += dt
        return qn[0]
    exact = 0.5 * (np.cos(1) + np.sin(1)) + 0.5 * np.exp(-1)
    e = [abs(solve(n) - exact) for n in (10, 20, 40)]
    order = np.log2(e[0] / e[1]), np.log2(e[1] / e[2])
    assert min(order) > 2.8


# ---------------------------------------------------------------- manufactured
class Sep:
    """f(x, y, z) = X(x) Y(y) Z(z) with analytic first derivatives."""

    def __init__(self, amp, X, dX, Y, dY, Z, dZ):
        self.a, self.X, self.dX, self.Y, self.dY, self.Z, self.dZ = amp, X, dX, Y, dY, Z, dZ

    def val(self, x, y, z):
        return self.a * self.X(x) * self.Y(y) * self.Z(z)

    def grad(self, x, y, z):
        X, Y, Z = self.X(x), self.Y(y), self.Z(z)
        return (self.a * self.dX(x) * Y * Z, self.a * X * self.dY(y) * Z,
                self.a * X * Y * self.dZ(z))


def manufactured(L, H):
    k = 2 * np.pi / L
    s, c_ = np.sin, np.cos
    one = lambda t: np.ones_like(t)
    zero = lambda t: np.zeros_like(t)
    return [
        Sep(2e-3, lambda x: c_(k * x), lambda x: -k * s(k * x),
            lambda y: s(k * y), lambda y: k * c_(k * y),
            lambda z: np.exp(-z / H), lambda z: -np.exp(-z / H) / H),
        Sep(6.0, lambda x: s(k * x), lambda x: k * c_(k * x),
            lambda y: c_(k * y), lambda y: -k * s(k * y),
            lambda z: 1 + z / H, lambda z: one(z) / H),
        Sep(4.0, lambda x: c_(k * x + 0.3), lambda x: -k * s(k * x + 0.3),
            lambda y: c_(k * y), lambda y: -k * s(k * y),
            lambda z: np.exp(-z / H), lambda z: -np.exp(-z / H) / H),
        Sep(0.3, lambda x: s(k * x), lambda x: k * c_(k * x),
            lambda y: s(k * y), lambda y: k * c_(k * y),
            lambda z: s(np.pi * z / H), lambda z: np.pi / H * c_(np.pi * z / H)),
        Sep(0.8, lambda x: c_(k * x), lambda x: -k * s(k * x),
            lambda y: c_(k * y - 0.5), lambda y: -k * s(k * y - 0.5),
            lambda z: (1 - z / H) ** 2, lambda z: -2 * (1 - z / H) / H),
    ]


def exact_rhs(c, xyz, F):
    """The perturbation equations of Section 2 with analytic derivatives."""
    x, y, z = xyz.T
    ph = c["phys"]
    g, Rd, cp, p00, f = ph["g"], ph["R_d"], ph["c_p"], ph["p00"], ph["f"]
    gam = cp / (cp - Rd)
    bg = cases.reference_state(c, z)
    rp, u, v, w, tp = (Fi.val(x, y, z) for Fi in F)
    G = [Fi.grad(x, y, z) for Fi in F]
    rho = bg["rho0"] + rp
    th = bg["theta0"] + tp
    drho = (G[0][0], G[0][1], bg["drho0dz"] + G[0][2])
    dth = (G[4][0], G[4][1], bg["dtheta0dz"] + G[4][2])
    p = p00 * (Rd * rho * th / p00) ** gam
    p0 = p00 * (Rd * bg["rho0"] * bg["theta0"] / p00) ** gam
    dp = [gam * p * (drho[i] / rho + dth[i] / th) for i in range(3)]
    dp[2] = dp[2] - gam * p0 * (bg["drho0dz"] / bg["rho0"] + bg["dtheta0dz"] / bg["theta0"])
    vel = (u, v, w)
    adv = lambda gi: u * gi[0] + v * gi[1] + w * gi[2]
    R = np.empty((5, x.size))
    R[0] = -sum(drho[i] * vel[i] + rho * G[1 + i][i] for i in range(3))
    R[1] = -adv(G[1]) - dp[0] / rho + f * v
    R[2] = -adv(G[2]) - dp[1] / rho - f * u
    R[3] = -adv(G[3]) - dp[2] / rho - (rp / rho) * g
    R[4] = -adv(G[4]) - w * bg["dtheta0dz"]
    return R


def mms_error(N, nx, nz, refine_box=False):
    L, H = 100e3, 10e3
    if refine_box:
        cols = columns.refine_where(nx, nx, L, L, 1,
                                    lambda X, Y, l: (np.abs(X) < 0.2 * L) & (np.abs(Y) < 0.3 * L),
                                    samples=3)
    else:
        cols = columns.uniform(nx, nx)
    c = cases.get("vortex_8x8x4_n4")
    c.update(N=N, nx0=nx, ny0=nx, Lx=L, Ly=L, z_edges=np.linspace(0, H, nz + 1), columns=cols)
    m = build(c)
    F = manufactured(L, H)
    xyz = m.node_xyz
    q = np.stack([Fi.val(*xyz.T) for Fi in F])
    R = assembly.rhs(m, q, ref_local(c, m), c["phys"])
    Rex = exact_rhs(c, xyz, F)
    Rex[3, m.lid] = 0.0
    scale = np.abs(Rex).max(axis=1)
    return (np.abs(R - Rex).max(axis=1) / scale).max()


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("nc", [False, True])
def test_manufactured_h_convergence(N, nc):
    e = [mms_error(N, nx, nz, nc) for nx, nz in ((4, 2), (8, 4), (16, 8))]
    order = np.log2(e[1] / e[2])
    assert order > N - 0.5, (e, order)


def test_manufactured_spectral_in_N():
    e = [mms_error(N, 4, 2) for N in (2, 4, 6, 8)]
    assert all(e[i + 1] < 0.2 * e[i] for i in range(3)), e
    assert e[-1] < 1e-4 * e[0]


# ---------------------------------------------------------------- AMR flags
def test_flags_brute_force_against_prose():
    """Every small combination of node values, level and thresholds."""
    vals = [0.0, 1.0, 2.0, 3.0]
    thr_sets = [[0.5], [0.5, 2.5], [1.0, 1.0, 2.0], [1.5, 2.5, 2.5]]
    for thr in thr_sets:
        lvl_max = len(thr)
        combos = list(itertools.product(vals, repeat=3))
        for lvl in range(lvl_max + 1):
            C = np.array(combos)
            flags = amr.element_flags(C, np.full(len(combos), lvl), thr, lvl_max)
            for e, nodes in enumerate(combos):
                # Section 4.1: any node above threshold(lvl+1) and lvl < lvl_max
                refine = lvl < lvl_max and any(ck > thr[lvl] for ck in nodes)
                # every node at or below threshold(lvl) and lvl > 0
                coarsen = lvl > 0 and all(ck <= thr[lvl - 1] for ck in nodes)
                assert not (refine and coarsen)
                exp = 1 if refine else (-1 if coarsen else 0)
                assert flags[e] == exp


def test_flags_reject_decreasing_thresholds():
    with pytest.raises(ValueError):
        amr.element_flags(np.zeros((1, 2)), [0], [2.0, 1.0], 2)


def test_column_rule():
    cols = np.array([[1, 0, 0], [1, 1, 0], [1, 0, 1], [1, 1, 1], [0, 1, 0]])
    nz = 2
    ef = np.array([-1, -1, -1, -1, -1, -1, -1, -1, 0, 1])
    out = amr.column_flags(ef, cols, nz)
    assert list(out) == [-1, -1, -1, -1, 1]
    ef2 = ef.copy()
    ef2[3] = 0       # one element of sibling 1 keeps -> nobody in the family coarsens
    out2 = amr.column_flags(ef2, cols, nz)
    assert list(out2) == [0, 0, 0, 0, 1]


def test_fp32_mode_is_float32_arithmetic():
    """The oracle's reduced-precision mode really rounds to float32: its
    tendency differs from FP64 by float32 round-off amplified by the
    derivatives (between 1e-9 and 1e-3 relative per field); the hydrostatic
    rest stays at rest in both modes (every perturbation term vanishes)."""
    import numpy as np
    from harness import oracle_mesh, oracle_reference_local
    from oracle import assembly, metrics
    from synth import cases
    c = cases.get("vortex_8x8x4_n4")
    m = oracle_mesh(c)
    ref = oracle_reference_local(c, m)
    q = cases.initial_state(c, m.node_xyz)
    r64 = assembly.rhs(m, q, ref, c["phys"])
    r32 = assembly.rhs(m, q, ref, c["phys"], dtype=np.float32)
    err = metrics.rel_l2(r32, r64, metrics.RHS_FLOORS)
    assert np.all(err > 1e-9) and np.all(err < 1e-3), err
    rest = np.zeros_like(q)
    assert np.abs(assembly.rhs(m, rest, ref, c["phys"])).max() == 0.0
    r = assembly.rhs(m, rest, ref, c["phys"], dtype=np.float32)
    assert np.abs(r).max() < 1e-4


def _isothermal_split(case, m, T0=250.0):
    """Constant-N hydrostatic atmosphere written as perturbations about an
    isothermal hydrostatic reference (both satisfy the equation of state)."""
    import numpy as np
    from synth import atmosphere
    p = case["phys"]
    Rd, cp, g, p00 = p["R_d"], p["c_p"], p["g"], p["p00"]
    b = case["background"]

    def iso(z):
        pr = p00 * np.exp(-g * z / (Rd * T0))
        th = T0 * (p00 / pr) ** (Rd / cp)
        return dict(rho0=pr / (Rd * T0), theta0=th, dtheta0dz=th * g / (cp * T0))
    zl = m.zl
    ref = iso(zl)
    zg = m.node_xyz[:, 2]
    st = atmosphere.background(zg, b["theta_s"], b["N_bv"], g, Rd, cp, p00)
    rg = iso(zg)
    q = np.zeros((5, m.n_dof))
    q[0] = st["rho0"] - rg["rho0"]
    q[4] = st["theta0"] - rg["theta0"]
    return q, ref


def test_balanced_state_about_other_reference_converges_spectrally():
    """A hydrostatic state split about a different hydrostatic reference is
    steady in the continuum; discretely only R_w is nonzero (the other
    components are round-off: at rest with horizontally uniform fields their
    terms vanish), and it decays spectrally with the order N."""
    import numpy as np
    from harness import oracle_mesh
    from oracle import assembly
    from synth import cases
    res = []
    for N in range(2, 9):
        c = cases.get("small_uniform", N=N)
        m = oracle_mesh(c)
        q, ref = _isothermal_split(c, m)
        R = assembly.rhs(m, q, ref, c["phys"])
        assert np.abs(R[[0, 1, 2, 4]]).max() <= 1e-12     # round-off only
        res.append(np.abs(R[3]).max())
    res = np.array(res)
    assert res[0] > 1e-4                       # the split is not trivially balanced
    assert np.all(np.diff(np.log(res[1:])) < 0)  # monotone decay from N = 3
    assert res[-1] < 1e-6 * res[0]
