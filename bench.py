"""Throughput benchmark of the spectral-element stage on one MI355X.

A step is one explicit Runge-Kutta stage of the full hot path (hanging-point
interpolation, element right-hand side, direct stiffness summation with the
hanging-node gather, inverse mass, lid rule and stage update) on the
64 x 64 x 16-element, N = 4 synthetic vortex workload (4,259,840 unique GLL
nodes, 8,192,000 local points), stages cycling through the three SSP-RK3
stages.  Prints one JSON line.

value    : unique GLL DOF-stage updates per second (n_dof * steps / time)
roofline : HBM roofline of the fused stage kernel, algorithmic bytes
           80 B (stage 1) or 120 B (stages 2, 3) per unique node per stage
           over the kernel time measured with HIP events on its stream
cpu_baseline : the FP64 oracle on the host, one stage of the same workload
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "vortex_64x64x16_n4"
METRIC = "GLL DOF-stage updates/s + AMR wall-time speedup at matched max-wind error"


def algorithmic_bytes(n_dof, stage):
    """Minimum HBM bytes of one stage: read q^n (and q_s) and write q_out."""
    return n_dof * (80 if stage == 0 else 120)


def cpu_baseline(case, n_stages=1):
    """Time the oracle (as it stands) on one stage of the same workload."""
    import numpy as np
    from oracle import assembly, timestep
    from oracle.mesh import OracleMesh
    from synth import cases
    om = OracleMesh(case["N"], case["nx0"], case["ny0"], case["Lx"], case["Ly"], case["z_edges"],
                    case["columns"], case["periodic_x"], case["periodic_y"])
    q0 = cases.initial_state(case, om.node_xyz)
    bl = cases.reference_state(case, om.zl)
    ref = dict(rho0=bl["rho0"], theta0=bl["theta0"], dtheta0dz=bl["dtheta0dz"])
    t = time.perf_counter()
    timestep.run_stages(lambda q: assembly.rhs(om, q, ref, case["phys"]), q0, case["dt"], n_stages)
    el = time.perf_counter() - t
    return {"value": om.n_dof * n_stages / el, "unit": "DOF-stage/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_stages} SSP-RK3 stage(s) of {WORKLOAD} (full mesh, {om.n_dof} unique "
                      f"nodes), single-threaded NumPy/SciPy, mesh setup not timed; {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU column "
              "partition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"

    import numpy as np
    import torch
    from paper_2410_21607_amd import api
    from oracle.timestep import stage_coefficients  # coefficients only (a, b, c)
    from synth import cases

    dev = torch.device("cuda:0")
    case = cases.get(WORKLOAD)
    mesh = api.Mesh.from_case(case)
    _, _, z = mesh.coords()
    bg = cases.reference_state(case, z)
    mesh.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    q0 = cases.initial_state(case, mesh.node_xyz())
    prec = api.SEM_FP64 if args.precision == "fp64" else api.SEM_FP32
    qn = torch.tensor(q0.reshape(-1), dtype=torch.float64, device=dev)
    qs = qn.clone()
    out = torch.empty_like(qn)
    n_dof = mesh.n_dof
    stream = torch.cuda.current_stream()

    def run(n, start_stage, events=None):
        nonlocal qs, out
        for i in range(n):
            s = (start_stage + i) % 3
            a, b, c = stage_coefficients(s, case["dt"])
            if events is not None:
                events[i][0].record(stream)
            api.sem_stage(mesh, a, b, c, qn, qs, out, prec)
            if events is not None:
                events[i][1].record(stream)
            qs, out = out, qs
            if s == 2:
                qn.copy_(qs)
        return start_stage + n

    st = run(args.warmup, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_timed = st
    st = run(args.steps, st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # kernel time of the stage launches, with HIP events on the launch stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    st2 = run(args.steps, st, ev)
    torch.cuda.synchronize()
    durs = np.array([a.elapsed_time(b) for a, b in ev]) * 1e-3
    stages = [(st + i) % 3 for i in range(args.steps)]
    alg = np.array([algorithmic_bytes(n_dof, s) for s in stages], dtype=np.float64)
    achieved = alg.sum() / durs.sum() / 1e9
    ok = bool(torch.isfinite(qs).all().item())
    del st2, st_timed

    res = {
        "metric": METRIC,
        "value": n_dof * args.steps / wall,
        "unit": "DOF-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == api.SEM_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "N": case["N"], "elements": int(mesh.info["n_elem"]),
                   "n_dof": int(n_dof), "local_points": int(mesh.n_local),
                   "step": "one SSP-RK3 stage (stages cycle 1,2,3)", "finite": ok},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sem_stage", "avg_kernel_ms": float(durs.mean() * 1e3)},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
