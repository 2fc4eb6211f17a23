"""Named synthetic workloads (inputs only).

Each case is a plain dict:
  N, nx0, ny0, Lx, Ly, z_edges, columns (n_col x 3 of level, ix, iy),
  periodic_x, periodic_y, phys (f, g, R_d, c_p, p00), background
  (theta_s, N_bv), vortex (v_max, r_max, z_top_v), noise (amp, z_top, seed),
  dt, stages.

Workloads (all doubly periodic with rigid lids, f-plane, constant N_bv=0.01,
theta_s=300 K):

* ``vortex_8x8x4_n4``     : 8 x 8 x 4 elements, N=4, 400 x 400 x 20 km,
                            V_max 15 m/s at 50 km, +-0.1 K noise everywhere,
                            dt 0.95 s, 10 stages (oracle runs in seconds).
* ``vortex_64x64x16_n4``  : 64 x 64 x 16 elements, N=4, 1000 x 1000 x 25 km,
                            V_max 25 m/s at 40 km, +-0.5 K noise below 2 km,
                            dt 0.29 s, 100 stages (throughput workload).
* ``amr2_64x64x8_n4`` / ``amr2_64x64x8_n7`` : 64 x 64 x 8 base on the
                            400 x 400 x 20 km domain, columns refined once where
                            the surface vertical vorticity of the vortex exceeds
                            2e-4 1/s; dt 0.48 s (N=4) / 0.18 s (N=7).
* ``share{2,4,8}_64x{32,16,8}x16_n4`` : one GPU's share of ``vortex_64x64x16_n4``
                            split 2, 4 or 8 ways along y (a strip, periodic in
                            x only).
* small meshes for tests (``small_*``).

The time steps follow dt = 0.4 h_min / (c_s + |u|_max) with h_min the
smallest vertical node spacing and c_s ~ 347 m/s at the surface.
"""

import numpy as np

from . import atmosphere, columns

PHYS = dict(g=9.81, R_d=287.0, c_p=1004.0, p00=1.0e5)


def _case(N, nx0, ny0, Lx, Ly, H, n_z, cols, f=5e-5, v_max=15.0, r_max=50e3,
          z_top_v=15e3, noise_amp=0.1, noise_ztop=1e30, seed=0, dt=1.0,
          stages=10, periodic=True, theta_s=300.0, N_bv=0.01, name=""):
    phys = dict(PHYS)
    phys["f"] = float(f)
    return dict(name=name, N=int(N), nx0=int(nx0), ny0=int(ny0), Lx=float(Lx),
                Ly=float(Ly), z_edges=np.linspace(0.0, H, n_z + 1),
                columns=np.asarray(cols, dtype=np.int64),
                periodic_x=periodic, periodic_y=periodic, phys=phys,
                background=dict(theta_s=theta_s, N_bv=N_bv),
                vortex=dict(v_max=v_max, r_max=r_max, z_top_v=z_top_v),
                noise=dict(amp=noise_amp, z_top=noise_ztop, seed=seed),
                dt=float(dt), stages=int(stages))


def _vorticity_refiner(case, thresholds):
    vx = vortex_of(case)

    xc, yc = case["vortex"].get("center", (0.0, 0.0))

    def pred(x, y, level):
        if level >= len(thresholds):
            return np.zeros_like(x, dtype=bool)
        return vx.vorticity_surface(np.hypot(x - xc, y - yc)) > thresholds[level]
    return pred


def get(name, **over):
    if name == "vortex_8x8x4_n4":
        c = _case(4, 8, 8, 400e3, 400e3, 20e3, 4, columns.uniform(8, 8), v_max=15.0,
                  r_max=50e3, noise_amp=0.1, dt=0.95, stages=10, name=name)
    elif name == "vortex_64x64x16_n4":
        c = _case(4, 64, 64, 1000e3, 1000e3, 25e3, 16, columns.uniform(64, 64),
                  v_max=25.0, r_max=40e3, noise_amp=0.5, noise_ztop=2e3, dt=0.29,
                  stages=100, name=name)
    elif name in ("share2_64x32x16_n4", "share4_64x16x16_n4", "share8_64x8x16_n4"):
        # one GPU's share of the 64 x 64 x 16 workload split k ways along y:
        # a 64 x (64/k) x 16 strip, periodic in x only (its y faces would
        # border the neighbouring GPUs' strips)
        k = int(name[5])
        ny = 64 // k
        c = _case(4, 64, ny, 1000e3, 1000e3 / k, 25e3, 16, columns.uniform(64, ny),
                  v_max=25.0, r_max=40e3, noise_amp=0.5, noise_ztop=2e3, dt=0.29,
                  stages=100, name=name)
        c["periodic_y"] = False
    elif name in ("amr2_64x64x8_n4", "amr2_64x64x8_n7"):
        N = 4 if name.endswith("n4") else 7
        c = _case(N, 64, 64, 400e3, 400e3, 20e3, 8, columns.uniform(64, 64),
                  v_max=15.0, r_max=50e3, noise_amp=0.1,
                  dt=0.48 if N == 4 else 0.18, stages=10, name=name)
        pred = _vorticity_refiner(c, [2e-4])
        c["columns"] = columns.refine_where(64, 64, 400e3, 400e3, 1, pred)
    elif name.startswith("small_uniform"):
        # small_uniform[_nN]: 4 x 3 x 3 elements, ragged aspect ratios
        N = int(over.pop("N", 4))
        c = _case(N, 4, 3, 400e3, 300e3, 20e3, 3, columns.uniform(4, 3),
                  v_max=15.0, r_max=60e3, noise_amp=0.1, dt=0.95, stages=4, name=name)
    elif name.startswith("small_amr2"):
        # 6 x 6 x 2 base, a 2 x 3 block of columns refined once
        N = int(over.pop("N", 4))
        periodic = bool(over.pop("periodic", True))
        c = _case(N, 6, 6, 400e3, 400e3, 20e3, 2, columns.uniform(6, 6),
                  v_max=15.0, r_max=60e3, noise_amp=0.1, dt=0.5, stages=4,
                  periodic=periodic, name=name)
        sel = {(2, 2), (3, 2), (2, 3), (3, 3), (2, 4), (3, 4)}
        c["columns"] = columns.refine_to_target(
            6, 6, lambda l, x, y: 1 if (l == 0 and (x, y) in sel) else l, 1, periodic)
    elif name.startswith("small_amr3"):
        # 4 x 4 x 2 base, two refinement levels around one corner (2:1 balanced)
        N = int(over.pop("N", 4))
        periodic = bool(over.pop("periodic", True))
        c = _case(N, 4, 4, 400e3, 400e3, 20e3, 2, columns.uniform(4, 4),
                  v_max=15.0, r_max=60e3, noise_amp=0.1, dt=0.3, stages=4,
                  periodic=periodic, name=name)

        def tgt(l, x, y):
            # refine level-0 cell (1,1) and (2,1); then the level-1 child (3,3)
            if l == 0 and (x, y) in {(1, 1), (2, 1)}:
                return 1
            if l == 1 and (x, y) == (3, 3):
                return 2
            return l
        c["columns"] = columns.refine_to_target(4, 4, tgt, 2, periodic)
    elif name.startswith("vortex3_64x64x8_n4") or name.startswith("small_vortex3"):
        # three-level AMR workload around a translating vortex: 40 m/s at
        # 25 km, uniform steering wind, seeded theta noise; layout refined by
        # the analytic surface vorticity at thresholds 2e-4 and 1e-3 s-1
        small = name.startswith("small")
        nb, nz = (16, 4) if small else (64, 8)
        seed = int(over.pop("seed", 0))
        c = _case(4, nb, nb, 400e3, 400e3, 20e3, nz, columns.uniform(nb, nb), v_max=40.0,
                  r_max=25e3, noise_amp=0.1, seed=seed, dt=0.85 if small else 0.27,
                  stages=10, name=name)
        c["steer"] = (10.0, 0.0)
        c["amr"] = dict(criterion=1, thresholds=[2e-4, 1e-3], lvl_max=2, interval=100)
        # a smooth profile (no vorticity jump at r_max) and smooth seeded
        # perturbations: an inviscid run stays free of grid-scale noise; the
        # seed also moves the vortex centre by up to 10 km
        c["vortex"]["profile"] = "smooth"
        rs = np.random.default_rng(1000 + seed)
        c["vortex"]["center"] = tuple(rs.uniform(-10e3, 10e3, size=2))
        c["noise"] = dict(amp=0.3, z_top=1e30, seed=seed, kind="modes")
        pred = _vorticity_refiner(c, c["amr"]["thresholds"])
        c["columns"] = columns.refine_where(nb, nb, 400e3, 400e3, 2, pred)
    elif name.startswith("tstar_64x64x8_n4"):
        # time-to-solution study: the smooth 40 m/s vortex on the 400 km
        # domain (at rest unless `steer` is given), refined by wind speed
        # with the paper's thresholds (7.5 m/s per level); `level` picks the
        # layout: uniform at that level, or the speed-refined layout up to
        # that level (`amr`)
        seed = int(over.pop("seed", 0))
        level = int(over.pop("level", 0))
        amr = bool(over.pop("amr", False))
        c = _case(4, 64, 64, 400e3, 400e3, 20e3, 8, columns.uniform(64, 64), v_max=40.0,
                  r_max=25e3, noise_amp=0.3, seed=seed, dt=0.43, stages=10, name=name)
        c["vortex"]["profile"] = "smooth"
        c["noise"] = dict(amp=0.3, z_top=1e30, seed=seed, kind="modes")
        thr = [7.5, 15.0, 22.5, 30.0][:max(level, 1)]
        c["amr"] = dict(criterion=0, thresholds=thr, lvl_max=level, interval=100)
        # stable step of the finest level present (vertical spacing limits levels 0-1)
        c["dt"] = {0: 0.43, 1: 0.43, 2: 0.27, 3: 0.135, 4: 0.0675}[level]
        # optional uniform steering wind (m/s): the vortex translates
        c["steer"] = tuple(over.pop("steer", (0.0, 0.0)))
        if amr and level > 0:
            vx = vortex_of(c)

            def pred(x, y, l):
                if l >= level:
                    return np.zeros_like(x, dtype=bool)
                return vx.vt_surface(np.hypot(x, y)) > thr[l]
            c["columns"] = columns.refine_where(64, 64, 400e3, 400e3, level, pred)
        elif level > 0:
            n = 64 << level
            cols = np.array([(level, x, y) for x in range(n) for y in range(n)])
            c["columns"] = columns.morton_sort(cols, level)
    else:
        raise KeyError(name)
    for k, v in over.items():
        c[k] = v
    return c


def vortex_of(case):
    v = case["vortex"]
    L = min(case["Lx"], case["Ly"])
    return atmosphere.Vortex(v["v_max"], v["r_max"], L / 4.0, L / 2.0, v["z_top_v"],
                             case["phys"]["f"], profile=v.get("profile", "rankine"))


def reference_state(case, z):
    b = case["background"]
    p = case["phys"]
    return atmosphere.background(z, b["theta_s"], b["N_bv"], p["g"], p["R_d"],
                                 p["c_p"], p["p00"])


def initial_state(case, xyz, vortex=None):
    if vortex is None:
        vortex = vortex_of(case)
    nz = case["noise"]
    bg = lambda z: reference_state(case, z)
    q = atmosphere.initial_state(np.asarray(xyz, dtype=np.float64), bg, vortex,
                                 case["phys"], nz["amp"], nz["z_top"], nz["seed"],
                                 case["Lx"], case["Ly"],
                                 center=case["vortex"].get("center", (0.0, 0.0)),
                                 noise_kind=nz.get("kind", "nodes"))
    su, sv = case.get("steer", (0.0, 0.0))
    if su or sv:
        # uniform steering wind over the vortex (the lids keep w = 0)
        q[1] += su
        q[2] += sv
    return q
