"""Throughput benchmark of the spectral-element stage on one MI355X.

A step is one explicit Runge-Kutta stage of the full hot path (hanging-point
interpolation, element right-hand side, direct stiffness summation with the
hanging-node gather, inverse mass, lid rule and stage update) on the
64 x 64 x 16-element, N = 4 synthetic vortex workload (4,259,840 unique GLL
nodes, 8,192,000 local points), stages cycling through the three SSP-RK3
stages.  Prints one JSON line.

value    : unique GLL DOF-stage updates per second (n_dof * steps / time)
roofline : HBM roofline of the fused stage, algorithmic bytes 80 B (stage 1)
           or 120 B (stages 2, 3) per unique node per stage, over the kernel
           time measured with HIP events around each captured RK3 step on the
           stream it replays on; `traffic` is the HBM bytes per stage read from
           the committed rocprofv3 counter summary when it matches the kernel
           source, else null
cpu_baseline : the FP64 oracle on the host cores, timed before any GPU call
               (one thread and all cores; this workload at 3 stages and the
               8 x 8 x 4 workload at 10 stages)
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "vortex_64x64x16_n4"
# names of the sem_stage work layouts (SEM_LAYOUT_COLUMNS, _BLOCKS, _COLUMNS_KZ, _COLUMNS_SPLIT)
LAYOUT_NAMES = {0: "columns", 1: "blocks", 2: "columns_kz", 3: "columns_split"}
METRIC = "GLL DOF-stage updates/s + AMR wall-time speedup at matched max-wind error"


def algorithmic_bytes(n_dof, stage):
    """Minimum HBM bytes of one stage: read q^n (and q_s) and write q_out."""
    return n_dof * (80 if stage == 0 else 120)


def cpu_baseline(plan=(("vortex_8x8x4_n4", 10), (WORKLOAD, 3))):
    """Time the oracle (as it stands, never tuned) on the host cores before
    any GPU call: for every (workload, stages) of the plan, the stages once
    with the BLAS/OpenMP pools at one thread and once at every core of this
    process's affinity mask.  The mesh and initial state are built once per
    workload and not timed.  value = the bench workload's rate with all
    cores; each leg also reports process CPU time over wall time, the
    parallelism the oracle actually reached."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import assembly, timestep
    from oracle.mesh import OracleMesh
    from synth import cases
    n_cores = len(os.sched_getaffinity(0))
    legs = []
    for name, n_stages in plan:
        case = cases.get(name)
        om = OracleMesh(case["N"], case["nx0"], case["ny0"], case["Lx"], case["Ly"], case["z_edges"],
                        case["columns"], case["periodic_x"], case["periodic_y"])
        q0 = cases.initial_state(case, om.node_xyz)
        bl = cases.reference_state(case, om.zl)
        ref = dict(rho0=bl["rho0"], theta0=bl["theta0"], dtheta0dz=bl["dtheta0dz"])
        for threads in (1, n_cores):
            with threadpool_limits(limits=threads):
                w0, c0 = time.perf_counter(), time.process_time()
                timestep.run_stages(lambda q: assembly.rhs(om, q, ref, case["phys"]), q0, case["dt"],
                                    n_stages)
                wall, cpu = time.perf_counter() - w0, time.process_time() - c0
            legs.append({"workload": name, "n_dof": int(om.n_dof), "stages": n_stages,
                         "threads": threads, "seconds": wall,
                         "dof_stage_per_s": om.n_dof * n_stages / wall,
                         "ms_per_stage": wall / n_stages * 1e3,
                         "cpu_time_over_wall": cpu / wall})
            print(f"  cpu baseline {name}: {n_stages} stages, {threads} thread(s): {wall:.1f} s",
                  file=sys.stderr, flush=True)
        del om, q0, bl, ref
    main = [g for g in legs if g["workload"] == WORKLOAD and g["threads"] == n_cores][-1]
    return {"value": main["dof_stage_per_s"], "unit": "DOF-stage/s", "cores": n_cores,
            "kind": "oracle",
            "sample": f"{main['stages']} SSP-RK3 stages of {WORKLOAD} (full mesh, {main['n_dof']} unique "
                      f"nodes) with the BLAS/OpenMP pools at {n_cores} threads (the affinity mask); "
                      f"mesh set-up not timed; the oracle's NumPy/SciPy steps ran at "
                      f"{main['cpu_time_over_wall']:.2f} CPU-seconds per second; legs lists both "
                      f"thread settings and the 8x8x4 workload at 10 stages",
            "legs": legs}


def kernel_source_hash():
    """Hash of the fused-stage kernel source (to detect stale counter data)."""
    h = hashlib.sha256()
    for f in ("stage_fused.hip", "stage_fused.h", "devmesh.h"):
        with open(os.path.join(ROOT, "paper_2410_21607_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload=WORKLOAD, kernel=None):
    """HBM bytes per stage from the committed rocprofv3 counter summary, or
    None when it is missing, was taken on a different kernel source, or (when
    `kernel` names the instance timed, e.g. "k_stage_columns<5, 4, double,
    false, false, 1>") on another instance."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    # one record per counted instance (a single record in older files)
    for rec in t.get("records", [t]):
        if rec.get("kernel_source_hash") != kernel_source_hash():
            continue
        if kernel is not None and kernel not in rec.get("kernel", ""):
            continue
        return rec.get("hbm_bytes_per_stage")
    return None


def column_instance(N, lpc, layout, fp64, diss_inline):
    """Name of the column-kernel instance a stage runs (template arguments:
    N + 1, layers per chunk, precision, terrain, dissipation, thread order),
    or None for the block layout."""
    order = {0: 0, 2: 1, 3: 2}.get(layout)
    if order is None:
        return None
    if not fp64:
        order = 1
    return (f"k_stage_columns<{N + 1}, {lpc}, {'double' if fp64 else 'float'}, false, "
            f"{'true' if diss_inline else 'false'}, {order}>")


def traffic_from_counters(fetch_csv, write_csv, workload=WORKLOAD, launches_per_stage=4, out_dir=None):
    """Write profiles/traffic_<workload>.json from two rocprofv3 counter runs
    of ``bench.py --copy-calibration`` on this workload: ``--pmc FETCH_SIZE``
    then ``--pmc WRITE_SIZE`` (KiB per dispatch).  Each counter is scaled by
    what it reads for the calibration kernel (torch's elementwise multiply,
    which reads and writes one state-sized array of known size); the column
    kernel's figure is the median per dispatch of its most frequent instance
    (the one the bench times) times the launches of one stage (four colours on
    a uniform periodic mesh).  Runs on the host only."""
    import csv
    import statistics
    import numpy as np
    from paper_2410_21607_amd import api
    from synth import cases
    case = cases.get(workload)
    if int(np.asarray(case["columns"])[:, 0].max()) != 0:
        raise ValueError("the traffic summary covers uniform meshes only")
    info = api.sem_mesh_plan(case)[0]
    calib_bytes = 5 * info["n_h"] * info["ldz"] * 8

    def per_kernel(path, counter):
        vals = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals
    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    # the multiply is the most frequent elementwise kernel of such a run
    calib = [k for k in fetch if "elementwise_kernel" in k and "Unary" in k]
    cols = [k for k in fetch if "k_stage_columns" in k]
    if not calib or not cols:
        raise ValueError("counter files hold no calibration kernel or no column kernel")
    calib_k = max(calib, key=lambda k: len(fetch[k]))
    main_k = max(cols, key=lambda k: len(fetch[k]))
    main_w = max((k for k in write if "k_stage_columns" in k), key=lambda k: len(write[k]), default=None)
    if main_w != main_k:
        raise ValueError("the FETCH_SIZE and WRITE_SIZE runs timed different column kernels "
                         f"({main_k} / {main_w}); pin the layout with --layout")
    f_fac = calib_bytes / (statistics.median(fetch[calib_k]) * 1024)
    w_fac = calib_bytes / (statistics.median(write[calib_k]) * 1024)
    f_kib, w_kib = statistics.median(fetch[main_k]), statistics.median(write[main_k])
    per_stage = launches_per_stage * 1024 * (f_kib * f_fac + w_kib * w_fac)
    out = {"kernel_source_hash": kernel_source_hash(), "kernel": main_k,
           "launches_per_stage": launches_per_stage, "hbm_bytes_per_stage": per_stage,
           "fetch_kib_per_launch": f_kib, "write_kib_per_launch": w_kib,
           "fetch_factor": f_fac, "write_factor": w_fac, "calibration_bytes": calib_bytes,
           "dispatches": len(fetch[main_k]),
           "source": f"profiles/fused_stage_{workload}.md"}
    # kept beside the records of other instances taken on the same sources
    path = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"traffic_{workload}.json")
    records = []
    if os.path.exists(path):
        with open(path) as fh:
            old = json.load(fh)
        records = [r for r in old.get("records", [old])
                   if r.get("kernel_source_hash") == out["kernel_source_hash"] and r.get("kernel") != main_k]
    with open(path, "w") as fh:
        json.dump({"records": records + [out]}, fh, indent=1)
    return out


def prepare(case_name, device):
    import torch  # noqa: F401
    from paper_2410_21607_amd import api
    from synth import cases
    case = cases.get(case_name)
    mesh = api.Mesh.from_case(case)
    _, _, z = mesh.coords()
    bg = cases.reference_state(case, z)
    mesh.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    q0 = mesh.unpack(cases.initial_state(case, mesh.node_xyz()), device=device)
    return case, mesh, q0


def timed_run(mesh, q0, dt, prec, n_steps):
    """Autotune, capture, warm up, then time n_steps RK3 steps; returns
    (seconds per stage, final state)."""
    import torch
    from paper_2410_21607_amd import api
    from paper_2410_21607_amd.solver import Stepper
    scratch = torch.zeros_like(q0)
    api.sem_stage_autotune(mesh, q0, q0.clone(), scratch, prec, reps=3)
    del scratch
    st = Stepper(mesh, q0, dt, prec, graph=True)
    st.step(1)
    torch.cuda.synchronize()
    st.buf[0].copy_(q0)
    st.cur = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.step(n_steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / (3 * n_steps), st.q


def fp32_variant(case, mesh, q0, n_steps=334):
    """FP32 element arithmetic vs the FP64 path over 3*n_steps stages: per-field
    floor-scaled relative L2 and the maximum-wind deviation (|u_h| max within
    [-50, 50] km square, full depth)."""
    import numpy as np
    from paper_2410_21607_amd import api
    t64, q64 = timed_run(mesh, q0, case["dt"], api.SEM_FP64, n_steps)
    t32, q32 = timed_run(mesh, q0, case["dt"], api.SEM_FP32, n_steps)
    a, b = mesh.pack(q32), mesh.pack(q64)
    floors = np.array([1e-3, 1.0, 1.0, 1.0, 0.1])
    rel = [float(np.linalg.norm(a[f] - b[f]) / max(np.linalg.norm(b[f]), floors[f] * np.sqrt(a.shape[1])))
           for f in range(5)]
    xyz = mesh.node_xyz()
    sel = (np.abs(xyz[:, 0]) <= 50e3) & (np.abs(xyz[:, 1]) <= 50e3)
    vm = lambda q: float(np.sqrt(q[1, sel] ** 2 + q[2, sel] ** 2).max())
    return {"stages": 3 * n_steps, "rel_l2_vs_fp64": dict(zip(["rho_p", "u", "v", "w", "theta_p"], rel)),
            "vmax_fp64": vm(b), "vmax_fp32": vm(a), "vmax_rel_dev": abs(vm(a) - vm(b)) / vm(b),
            "ms_per_stage_fp64": t64 * 1e3, "ms_per_stage_fp32": t32 * 1e3,
            "note": "FP64 GPU trajectory as reference (it matches the FP64 oracle to <=1e-12 per "
                    "stage at this size, tested over 3 stages)"}


def amr_throughput(device):
    """Two-level AMR meshes (all levels and hanging faces in the same passes)
    against the uniform mesh at the finest level, per-stage cost."""
    import torch
    from synth import cases, columns
    from paper_2410_21607_amd import api
    out = {}
    for name in ("amr2_64x64x8_n4", "amr2_64x64x8_n7"):
        case, mesh, q0 = prepare(name, device)
        t, _ = timed_run(mesh, q0, case["dt"], api.SEM_FP64, 20)
        fine = dict(case)
        fine["nx0"], fine["ny0"] = 2 * case["nx0"], 2 * case["ny0"]
        fine["columns"] = columns.uniform(fine["nx0"], fine["ny0"])
        fm = api.Mesh.from_case(fine)
        _, _, z = fm.coords()
        bg = cases.reference_state(fine, z)
        fm.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
        fq = fm.unpack(cases.initial_state(fine, fm.node_xyz()), device=device)
        tf, _ = timed_run(fm, fq, case["dt"], api.SEM_FP64, 20)
        per_node = sum(algorithmic_bytes(1, s) for s in range(3)) / 3.0
        achieved = mesh.n_dof * per_node / t / 1e9
        out[name] = {"n_dof": int(mesh.n_dof), "n_col": int(mesh.info["n_col"]),
                     "hanging_points": int(mesh.info["n_hh"]),
                     "dof_stage_per_s": mesh.n_dof / t, "ms_per_stage": t * 1e3,
                     "uniform_finest_ms_per_stage": tf * 1e3,
                     "cost_ratio_uniform_over_amr": tf / t,
                     "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                                  "algorithmic_bytes_per_node_stage": per_node,
                                  "note": "wall time of graph-replayed RK3 steps"}}
        del mesh, fm, q0, fq
        torch.cuda.empty_cache()
    return out


def terrain_throughput(device, flat_ms=None, case_name=WORKLOAD, amp=2000.0, half_width=60e3,
                       n_steps=20):
    """A workload over a Gaussian mountain (terrain-following coordinates):
    per-stage cost, and the roofline with the reference state read per node
    (five FP64 arrays, 40 B per node on top of the state)."""
    import numpy as np
    import torch
    from paper_2410_21607_amd import api
    from synth import cases
    case = cases.get(case_name)
    mesh = api.Mesh.from_case(case)
    hxy, _, zf = mesh.coords()
    zs = amp * np.exp(-(hxy[:, 0] ** 2 + hxy[:, 1] ** 2) / half_width ** 2)
    zp = mesh.heights(zs)
    bg = cases.reference_state(case, zp)
    mesh.set_terrain(zs, bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    xyz = mesh.node_xyz()
    xyz[:, 2] = zp
    q0 = mesh.unpack(cases.initial_state(case, xyz), device=device)
    t, q = timed_run(mesh, q0, case["dt"], api.SEM_FP64, n_steps)
    lpc64 = api.sem_stage_get_tune(mesh)
    # reduced precision over the same terrain: after the same number of stages,
    # the floor-scaled deviation from the FP64 run
    t32, q32 = timed_run(mesh, q0, case["dt"], api.SEM_FP32, n_steps)
    d32 = np.abs(mesh.pack(q32) - mesh.pack(q)).max(axis=1) / np.array([1e-3, 1.0, 1.0, 1.0, 0.1])
    fp32 = {"ms_per_stage": t32 * 1e3, "dof_stage_per_s": mesh.n_dof / t32,
            "layers_per_chunk": api.sem_stage_get_tune(mesh),
            "max_floor_scaled_deviation_from_fp64": [float(x) for x in d32],
            "stages": 3 * n_steps, "finite": bool(torch.isfinite(q32).all().item())}
    del q32
    per_node = sum(algorithmic_bytes(1, s) for s in range(3)) / 3.0 + 5 * 8
    achieved = mesh.n_dof * per_node / t / 1e9
    if flat_ms is None:
        # the same mesh with box elements, for the cost ratio
        fm = api.Mesh.from_case(case)
        bgf = cases.reference_state(case, zf)
        fm.set_reference(bgf["rho0"], bgf["theta0"], bgf["dtheta0dz"])
        fq = fm.unpack(cases.initial_state(case, fm.node_xyz()), device=device)
        tf, _ = timed_run(fm, fq, case["dt"], api.SEM_FP64, n_steps)
        flat_ms = tf * 1e3
        del fm, fq
    out = {"workload": case_name + " over a Gaussian mountain",
           "hanging_points": int(mesh.info["n_hh"]),
           "mountain": {"height_m": amp, "half_width_m": half_width},
           "n_dof": int(mesh.n_dof), "ms_per_stage": t * 1e3,
           "dof_stage_per_s": mesh.n_dof / t,
           "layers_per_chunk": lpc64,
           "algorithmic_bytes_per_node_stage": per_node,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS},
           "finite": bool(torch.isfinite(q).all().item()),
           "fp32": fp32}
    if flat_ms:
        out["cost_ratio_over_flat"] = t * 1e3 / flat_ms
    del mesh, q0, q
    torch.cuda.empty_cache()
    return out


def adaptive_run(case, device, forecaster=None, rebuild_every=1, recorder=None, adapt=True,
                 columns=None):
    """An AdaptiveRun of an AMR workload (``case["amr"]`` settings) from its
    synthetic initial state on the given (default: the case's) layout."""
    from paper_2410_21607_amd import api
    from paper_2410_21607_amd.adaptive import AdaptiveRun
    from synth import cases
    c = dict(case)
    if columns is not None:
        c["columns"] = columns
    mesh = api.Mesh.from_case(c)
    _, _, z = mesh.coords()
    bg = cases.reference_state(c, z)
    ref = (bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    mesh.set_reference(*ref)
    q0 = mesh.unpack(cases.initial_state(c, mesh.node_xyz()), device=device)
    a = c["amr"]
    return AdaptiveRun(mesh, q0, c["dt"], ref, a["criterion"], a["thresholds"], a["lvl_max"],
                       a["interval"], forecaster=forecaster, rebuild_every=rebuild_every,
                       on_boundary=recorder, adapt=adapt)


def project_to_level0(mesh, q):
    """The state projected onto the level-0 columns: finest-level sibling
    families are merged into their parents, one level at a time, with the
    library's transfer (the merge is the lumped-mass L2 projection of the four
    children).  Returns (mesh, state) on a Morton-ordered level-0 layout."""
    import numpy as np
    from paper_2410_21607_amd import api
    from synth import columns as sc
    cols = np.asarray(mesh.columns)
    while cols[:, 0].max() > 0:
        lm = int(cols[:, 0].max())
        keep = cols[cols[:, 0] < lm]
        fine = cols[cols[:, 0] == lm]
        parents = np.unique(np.stack([fine[:, 0] - 1, fine[:, 1] // 2, fine[:, 2] // 2], axis=1), axis=0)
        cols = sc.morton_sort(np.concatenate([keep, parents]), max(lm - 1, 0))
        new = mesh.with_columns(cols)
        out = new.state(device=q.device)
        api.sem_transfer_apply(api.Transfer(mesh, new), q, out)
        mesh, q = new, out
    return mesh, q


def projected_error(mesh_a, q_a, mesh_ref, q_ref):
    """Floor-scaled relative L2 per field (rho', u, v, w, theta'; floors 1e-3
    kg/m3, 1 m/s, 0.1 K) between two states after both are projected onto
    the level-0 columns (the same layout, so the same numbering)."""
    import numpy as np
    ma, pa = project_to_level0(mesh_a, q_a)
    mr, pr = project_to_level0(mesh_ref, q_ref)
    assert np.array_equal(np.asarray(ma.columns), np.asarray(mr.columns))
    a, b = ma.pack(pa), mr.pack(pr)
    floors = np.array([1e-3, 1.0, 1.0, 1.0, 0.1])
    return [float(np.linalg.norm(a[f] - b[f]) / max(np.linalg.norm(b[f]), floors[f] * np.sqrt(a.shape[1])))
            for f in range(5)]


def always_refine(run, plain_elem, plain_col):
    """Ablation of the forecaster: every column asks to be split."""
    import torch
    return torch.ones_like(plain_col)


def _summary(run, ref_vmax=None):
    import numpy as np
    v = np.array([b["vmax"] for b in run.log])
    out = {"wall_s": run.wall(), "step_s": run.timings["step"], "rebuilds": run.n_rebuild,
           "boundaries": run.n_boundary, "timings_s": dict(run.timings),
           "mean_n_dof": float(np.mean([b["n_dof"] for b in run.log])) if run.log else 0.0,
           "mean_split_flag_fraction": float(np.mean([b["split_frac"] for b in run.log]))
           if run.log else 0.0,
           "vmax_final": float(v[-1]) if v.size else None}
    if ref_vmax is not None and v.size:
        out["vmax_max_rel_dev_vs_uniform"] = float(np.max(np.abs(v - ref_vmax) / ref_vmax))
    return out


def forecaster_experiment(device, case_name="vortex3_64x64x8_n4", sim_seconds=405.0,
                          train_seeds=(0, 1, 2, 3, 4), eval_seeds=(5, 6, 7), horizon=5, n_samples=200000,
                          epochs=20):
    """Plain-criterion AMR vs forecaster-driven AMR vs the uniform finest mesh
    on a translating vortex: wall time and maximum-wind deviation."""
    import numpy as np
    import torch
    from paper_2410_21607_amd import forecast
    from synth import cases, columns as sc
    base = cases.get(case_name)
    n_steps = int(round(sim_seconds / base["dt"]))
    n_steps -= n_steps % base["amr"]["interval"]
    res = {"workload": case_name, "sim_seconds": n_steps * base["dt"], "steps": n_steps,
           "dt": base["dt"], "interval_steps": base["amr"]["interval"], "horizon_intervals": horizon,
           "thresholds": base["amr"]["thresholds"], "lvl_max": base["amr"]["lvl_max"],
           "steering_wind": base["steer"]}
    # 1. training data from plain-criterion runs
    X, Y = [], []
    t0 = time.perf_counter()
    for sd in train_seeds:
        rec = forecast.Recorder()
        run = adaptive_run(cases.get(case_name, seed=sd), device, recorder=rec)
        run.run(n_steps)
        x, y = rec.samples(horizon)
        X.append(x)
        Y.append(y)
        print(f"  training run seed {sd}: {len(y)} samples, {run.n_rebuild} rebuilds, "
              f"{run.wall():.1f} s", file=sys.stderr, flush=True)
        del run, rec
        torch.cuda.empty_cache()
    X, Y = np.concatenate(X), np.concatenate(Y)
    res["samples_available"] = int(Y.size)
    res["class_counts"] = np.bincount(Y, minlength=3).tolist()
    Xs, Ys = forecast.balanced_subset(X, Y, n_samples, seed=0)
    fc = forecast.Forecaster(seed=0, horizon=horizon)
    t1 = time.perf_counter()
    losses = fc.train(Xs, Ys, epochs=epochs, batch=1024, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    res["training"] = {"samples": int(Ys.size), "epochs": epochs, "loss_first": losses[0],
                       "loss_last": losses[-1], "train_s": time.perf_counter() - t1,
                       "collect_s": t1 - t0,
                       "accuracy_all_samples": float(np.mean(fc.predict(X) == Y))}
    del X, Y, Xs, Ys
    # 2. evaluation on unseen seeds
    per_seed = []
    for k, es in enumerate(eval_seeds):
        ev = cases.get(case_name, seed=es)
        lm = ev["amr"]["lvl_max"]
        fine = np.array([(lm, x, y) for x in range(ev["nx0"] << lm) for y in range(ev["ny0"] << lm)])
        uni = adaptive_run(ev, device, adapt=False, columns=sc.morton_sort(fine, lm))
        uni.run(n_steps)
        ref_v = np.array([b["vmax"] for b in uni.log])
        r = {"seed": es, "uniform_finest": _summary(uni)}
        torch.cuda.empty_cache()
        for key, kw in (("plain_amr", {}), ("plain_amr_sparse_rebuilds", {"rebuild_every": horizon}),
                        ("forecaster_amr", {"forecaster": fc, "rebuild_every": horizon}),
                        ("always_refine_sparse_rebuilds", {"forecaster": always_refine,
                                                           "rebuild_every": horizon})):
            run = adaptive_run(ev, device, **kw)
            run.run(n_steps)
            r[key] = _summary(run, ref_v)
            # under-resolution at the final time: the state against the uniform
            # finest run, both projected onto the level-0 columns
            r[key]["final_error_vs_uniform_l0_projection"] = projected_error(run.mesh, run.q, uni.mesh, uni.q)
            del run
            torch.cuda.empty_cache()
        del uni
        torch.cuda.empty_cache()
        if k == 0:
            # held-out skill: the seed's plain run, features at t vs classes at t + horizon
            rec = forecast.Recorder()
            chk = adaptive_run(ev, device, recorder=rec)
            chk.run(n_steps)
            Xe, Ye = rec.samples(horizon)
            res["heldout_scores"] = forecast.class_scores(fc.predict(Xe), Ye) if Ye.size else None
            del chk, rec
        p, f, u = r["plain_amr"], r["forecaster_amr"], r["uniform_finest"]
        r["speedup_forecaster_over_plain"] = p["wall_s"] / f["wall_s"]
        r["speedup_plain_amr_over_uniform"] = u["wall_s"] / p["wall_s"]
        r["speedup_forecaster_amr_over_uniform"] = u["wall_s"] / f["wall_s"]
        per_seed.append(r)
        print(f"  eval seed {es}: forecaster/plain {r['speedup_forecaster_over_plain']:.3f}", file=sys.stderr,
              flush=True)
    res["eval"] = per_seed
    agg = lambda key, sub: [r[key][sub] for r in per_seed]
    for key in ("plain_amr", "plain_amr_sparse_rebuilds", "forecaster_amr",
                "always_refine_sparse_rebuilds", "uniform_finest"):
        res[key] = {"wall_s_mean": float(np.mean(agg(key, "wall_s"))),
                    "rebuilds_mean": float(np.mean(agg(key, "rebuilds"))),
                    "mean_n_dof": float(np.mean(agg(key, "mean_n_dof"))),
                    "mean_split_flag_fraction": float(np.mean(agg(key, "mean_split_flag_fraction")))}
        if key != "uniform_finest":
            res[key]["vmax_max_rel_dev_vs_uniform"] = float(np.max(agg(key, "vmax_max_rel_dev_vs_uniform")))
            errs = np.array(agg(key, "final_error_vs_uniform_l0_projection"))
            res[key]["final_error_vs_uniform_l0_projection_mean"] = errs.mean(axis=0).tolist()
            res[key]["final_error_vs_uniform_l0_projection_max"] = errs.max(axis=0).tolist()
    for k2 in ("speedup_forecaster_over_plain", "speedup_plain_amr_over_uniform",
               "speedup_forecaster_amr_over_uniform"):
        v = [r[k2] for r in per_seed]
        res[k2] = float(np.mean(v))
        res[k2 + "_min"] = float(np.min(v))
    res["vmax_dev_difference"] = res["forecaster_amr"]["vmax_max_rel_dev_vs_uniform"] - \
        res["plain_amr"]["vmax_max_rel_dev_vs_uniform"]
    return res


def tstar_study(device, sim_seconds=60.0, max_level=4, full_uniform_level=3, steer=(10.0, 0.0),
                l4_steps=4):
    """Normalised time-to-solution T* = T / T(uniform level 0) of uniform
    meshes at levels 0..max_level and of AMR refined by wind speed up to each
    level (thresholds 7.5, 15, 22.5, 30 m/s for levels 1-4, the paper's set),
    on a vortex translating with a uniform steering wind, same simulated time.
    Uniform meshes above `full_uniform_level` are too large to initialise and
    run for the whole window: their T is the measured time of `l4_steps` RK3
    steps (HIP-graph replays, the same kernels; the rest state, since the
    kernel time does not depend on the values) times the window's steps.
    Maximum wind of each AMR run against the uniform run at its finest level
    (at the finest fully-run uniform level above that)."""
    import numpy as np
    import torch
    from paper_2410_21607_amd import api
    from paper_2410_21607_amd.solver import Stepper
    from synth import cases
    out = {"workload": "tstar_64x64x8_n4", "sim_seconds": sim_seconds, "steering_wind": list(steer),
           "thresholds": [7.5, 15.0, 22.5, 30.0][:max_level], "runs": {}}
    vref, base = {}, None
    for amr in (False, True):
        for lv in range(0 if not amr else 1, max_level + 1):
            c = cases.get("tstar_64x64x8_n4", level=lv, amr=amr, steer=steer)
            n = int(round(sim_seconds / c["dt"]))
            n -= n % c["amr"]["interval"]
            key = ("amr" if amr else "uniform") + f"_L{lv}"
            if not amr and lv > full_uniform_level:
                t0 = time.perf_counter()
                mesh = api.Mesh.from_case(c)
                _, _, z = mesh.coords()
                bg = cases.reference_state(c, z)
                mesh.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
                build_s = time.perf_counter() - t0
                st = Stepper(mesh, mesh.state(device=device), c["dt"], graph=True)
                st.step(1)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st.step(l4_steps)
                torch.cuda.synchronize()
                per_step = (time.perf_counter() - t1) / l4_steps
                rec = {"dt": c["dt"], "steps": n, "wall_s": per_step * n, "estimated": True,
                       "measured_steps": l4_steps, "s_per_step": per_step, "mesh_build_s": build_s,
                       "n_dof": int(mesh.n_dof), "n_col_start": int(len(c["columns"]))}
                del st, mesh
            else:
                run = adaptive_run(c, device, adapt=amr)
                run.run(n)
                torch.cuda.synchronize()
                v = np.array([b["vmax"] for b in run.log])
                tb = np.array([b["step"] for b in run.log]) * c["dt"]   # boundary times
                rec = {"dt": c["dt"], "steps": n, "wall_s": run.wall(), "rebuilds": run.n_rebuild,
                       "mean_n_dof": float(np.mean([b["n_dof"] for b in run.log])),
                       "n_col_start": int(len(c["columns"])), "vmax_final": float(v[-1]),
                       "timings_s": dict(run.timings)}
                if not amr:
                    vref[lv] = (tb, v)
                else:
                    # compare at the boundaries both runs share (equal simulated times)
                    ref_lv = min(lv, full_uniform_level)
                    tr, vr = vref[ref_lv]
                    common = [(i, j) for i in range(tb.size) for j in range(tr.size)
                              if abs(tb[i] - tr[j]) < 1e-6 * max(1.0, tr[j])]
                    ia, ir = (np.array(x) for x in zip(*common))
                    rec["vmax_reference_uniform_level"] = ref_lv
                    rec["vmax_compared_at_s"] = tr[ir].tolist()
                    rec["vmax_max_rel_dev_vs_uniform"] = float(np.max(np.abs(v[ia] - vr[ir]) / vr[ir]))
                del run
            if not amr and lv == 0:
                base = rec["wall_s"]
            rec["T_star"] = rec["wall_s"] / base
            out["runs"][key] = rec
            print(f"  {key}: {rec['wall_s']:.2f} s, T* {rec['T_star']:.2f}", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
    for lv in range(1, max_level + 1):
        out[f"speedup_amr_over_uniform_L{lv}"] = out["runs"][f"uniform_L{lv}"]["wall_s"] / \
            out["runs"][f"amr_L{lv}"]["wall_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300, help="RK stages to time (rounded up to whole RK3 steps)")
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--dissipation", default="",
                    help="Cs,sponge_gamma,sponge_depth: time the stage with the sub-grid and "
                         "absorbing-layer terms on (default off, the inviscid stage)")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="case timed for the main line (default: the 64x64x16 N=4 bench workload)")
    ap.add_argument("--layout", default="auto",
                    help="work layout of the timed stage: auto (the autotuner's choice), "
                         "columns:LAYERS_PER_CHUNK, columns_kz:LAYERS_PER_CHUNK (FP64 threads in "
                         "vertical-index order), columns_split:LAYERS_PER_CHUNK (a thread per element "
                         "and local node) or blocks:SEGMENTS")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP32-variant, AMR and forecaster measurements")
    ap.add_argument("--forecaster", action="store_true",
                    help="run the forecaster experiment even with --no-extras")
    ap.add_argument("--forecaster-only", action="store_true",
                    help="run only the forecaster experiment and print its JSON")
    ap.add_argument("--terrain-only", action="store_true",
                    help="run only the terrain-following measurement and print its JSON")
    ap.add_argument("--terrain-case", default="both",
                    help="with --terrain-only: a workload name, or both (the bench mesh and the "
                         "two-level AMR mesh)")
    ap.add_argument("--tstar-only", action="store_true",
                    help="run only the time-to-solution study (uniform vs AMR by level) and print its JSON")
    ap.add_argument("--tstar-seconds", type=float, default=60.0,
                    help="simulated seconds of each run of the time-to-solution study")
    ap.add_argument("--fc-case", default="vortex3_64x64x8_n4")
    ap.add_argument("--fc-seconds", type=float, default=405.0,
                    help="simulated seconds of each forecaster-experiment run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain device copies of the state size (counter calibration)")
    ap.add_argument("--traffic-from", default="",
                    help="FETCH_CSV,WRITE_CSV: write profiles/traffic_<workload>.json from the "
                         "counter files of two rocprofv3 --pmc runs (host only, no GPU) and exit")
    args = ap.parse_args()
    if args.traffic_from:
        fetch_csv, write_csv = args.traffic_from.split(",")
        print(json.dumps(traffic_from_counters(fetch_csv, write_csv, args.workload)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU column "
              "partition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)
    # the oracle's CPU baseline runs first, before anything touches the GPU
    cpu_base = None
    if not (args.no_cpu_baseline or args.terrain_only or args.tstar_only or args.forecaster_only):
        cpu_base = cpu_baseline()

    import numpy as np
    import torch
    from paper_2410_21607_amd import api
    from paper_2410_21607_amd.solver import Stepper
    from synth import cases

    dev = torch.device("cuda:0")
    if args.terrain_only:
        if args.terrain_case == "both":
            out = {"uniform": terrain_throughput(dev),
                   "two_level_amr": terrain_throughput(dev, case_name="amr2_64x64x8_n4")}
        else:
            out = terrain_throughput(dev, case_name=args.terrain_case)
        print(json.dumps(out), flush=True)
        return
    if args.tstar_only:
        print(json.dumps(tstar_study(dev, sim_seconds=args.tstar_seconds)), flush=True)
        return
    if args.forecaster_only:
        print(json.dumps(forecaster_experiment(dev, args.fc_case, args.fc_seconds)), flush=True)
        return
    case = cases.get(args.workload)
    mesh = api.Mesh.from_case(case)
    _, _, z = mesh.coords()
    bg = cases.reference_state(case, z)
    mesh.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    q0 = mesh.unpack(cases.initial_state(case, mesh.node_xyz()), device=dev)
    prec = api.SEM_FP64 if args.precision == "fp64" else api.SEM_FP32
    if args.dissipation:
        mesh.set_dissipation(*(float(x) for x in args.dissipation.split(",")))
    n_dof = mesh.n_dof
    if args.layout == "auto":
        scratch = torch.empty_like(q0)
        api.sem_stage_autotune(mesh, q0, q0.clone(), scratch, prec, reps=5)
        del scratch
    else:
        kind, par = args.layout.split(":")
        api.sem_stage_set_layout(mesh, {"columns": api.SEM_LAYOUT_COLUMNS,
                                        "columns_kz": api.SEM_LAYOUT_COLUMNS_KZ,
                                        "columns_split": api.SEM_LAYOUT_COLUMNS_SPLIT,
                                        "blocks": api.SEM_LAYOUT_BLOCKS}[kind], int(par))
    layout, layout_par = api.sem_stage_get_layout(mesh)
    lpc = api.sem_stage_get_tune(mesh)
    st = Stepper(mesh, q0, case["dt"], prec, graph=not args.no_graph)
    n_steps = max(1, -(-args.steps // 3))       # whole RK3 steps
    n_warm = max(1, -(-args.warmup // 3))
    st.step(n_warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.step(n_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # kernel time of each RK3 step with HIP events on the stream the graphs replay on
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n_steps)]
    for e0, e1 in ev:
        e0.record(stream)
        st.step(1)
        e1.record(stream)
    torch.cuda.synchronize()
    durs = np.array([a.elapsed_time(b) for a, b in ev]) * 1e-3
    alg_step = sum(algorithmic_bytes(n_dof, s) for s in range(3))
    achieved = alg_step / durs.mean() / 1e9
    ok = bool(torch.isfinite(st.q).all().item())
    # achievable streaming bandwidth for context: an elementwise kernel that
    # reads and writes one state-sized array (HIP events, mean of 20)
    src = torch.rand(mesh.n_state, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(20):
        torch.mul(src, 1.0, out=dst)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 20 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    if args.copy_calibration:
        # an elementwise kernel reading and writing one state-sized array
        # (5 n_dof doubles each way): the reference for HBM counter scaling
        src = torch.rand(mesh.n_state, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
    traffic = measured_traffic(args.workload, column_instance(
        case["N"], lpc, layout, prec == api.SEM_FP64,
        bool(args.dissipation) and prec == api.SEM_FP64 and layout != api.SEM_LAYOUT_BLOCKS))
    stages = 3 * n_steps
    res = {
        "metric": METRIC,
        "value": n_dof * stages / wall,
        "unit": "DOF-stage/s",
        "n_gpus": 1,
        "steps": stages,
        "warmup": 3 * n_warm,
        "ms_per_step": wall / stages * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == api.SEM_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": case["N"], "elements": int(mesh.info["n_elem"]),
                   "n_dof": int(n_dof), "local_points": int(mesh.n_local),
                   "step": "one SSP-RK3 stage (timed as HIP-graph replays of whole RK3 steps)",
                   "graph": not args.no_graph,
                   "layout": LAYOUT_NAMES[layout],
                   "layers_per_chunk" if layout != api.SEM_LAYOUT_BLOCKS else "segments":
                       lpc if layout != api.SEM_LAYOUT_BLOCKS else layout_par,
                   "finite": ok,
                   "dissipation": args.dissipation or "off"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "fused stage (column passes + hanging pass), per stage",
                     "copy_kernel_GBps": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs,
                     "avg_kernel_ms": float(durs.mean() * 1e3 / 3)},
    }
    if not args.no_extras:
        res["fp32_variant"] = fp32_variant(case, mesh, q0)
        res["amr_two_level"] = amr_throughput(dev)
        res["terrain"] = {"uniform": terrain_throughput(dev, flat_ms=res["ms_per_step"]),
                          "two_level_amr": terrain_throughput(dev, case_name="amr2_64x64x8_n4")}
    if args.forecaster or not args.no_extras:
        res["amr_forecaster"] = forecaster_experiment(dev, args.fc_case, args.fc_seconds)
    if cpu_base is not None:
        res["cpu_baseline"] = cpu_base
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
