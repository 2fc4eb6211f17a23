"""Dynamic h-adaptation driver (Section 4.1 and Algorithm 1 of the paper:
evaluate the refinement criterion, adapt the column quadtree, move the
solution, continue stepping).

Every ``interval`` RK3 steps the run reaches a boundary.  There:

1. ``amr_flag`` gives the criterion's element and column flags (+1 split,
   -1 merge, 0 keep) and ``sem_max_wind`` the intensity diagnostic;
2. an optional ``on_boundary(run, plain_elem)`` hook sees the state (data
   collection for the forecaster);
3. every ``rebuild_every``-th boundary the mesh may be rebuilt:
   a. optionally a forecaster (a callable taking the run and the criterion's
      flags and returning combined column flags on the device) replaces the
      column flags;
   b. ``sem_adapt_columns`` (host) gives the new layout (split, 2:1 balance,
      merge);
   c. a new mesh handle over it, its reference state (the vertical structure
      is unchanged, so the same per-level arrays are reused; over terrain the
      ``terrain`` hook gives the surface heights and the per-node reference of
      the new mesh), the transfer rows and one ``sem_transfer_apply`` launch;
   d. a new ``Stepper`` (HIP graphs recaptured for the new mesh).

The state at the previous boundary is kept on the current mesh
(``q_prev``) for the forecaster's rate-of-change features.  Wall time per
phase is accumulated in ``timings``; per-boundary diagnostics in ``log``.
"""

import time

import numpy as np
import torch

from . import api
from .solver import Stepper


def _same_layout(a, b):
    """True when two column layouts hold the same (level, ix, iy) set."""
    a, b = np.asarray(a, np.int64), np.asarray(b, np.int64)
    if a.shape != b.shape:
        return False
    rows = lambda c: c[np.lexsort((c[:, 2], c[:, 1], c[:, 0]))]
    return bool(np.array_equal(rows(a), rows(b)))


class AdaptiveRun:
    def __init__(self, mesh, q0, dt, reference, criterion, thresholds, lvl_max,
                 interval, precision=api.SEM_FP64, graph=True, layers_per_chunk=0,
                 forecaster=None, rebuild_every=1, on_boundary=None, wind_box=None,
                 adapt=True, terrain=None):
        """mesh: api.Mesh; q0: padded state tensor on it; reference: tuple of
        (rho0, theta0, dtheta0dz) per vertical node (already set on mesh);
        wind_box: (x0, x1, y0, y1) of the maximum-wind diagnostic (default:
        the whole domain); adapt=False keeps the mesh fixed (diagnostics only);
        terrain: optional callable mesh -> (zs per horizontal node, rho0,
        theta0, dtheta0dz per node), applied to every new mesh (the caller
        sets it on the first one).  The solution moves between layouts in the
        terrain-following coordinates."""
        self.mesh = mesh
        self.dt = float(dt)
        self.reference = tuple(np.asarray(a, dtype=np.float64) for a in reference)
        self.criterion = int(criterion)
        self.thresholds = np.asarray(thresholds, dtype=np.float64)
        self.lvl_max = int(lvl_max)
        self.interval = int(interval)
        self.precision = precision
        self.graph = bool(graph)
        self.lpc = int(layers_per_chunk)
        self.forecaster = forecaster
        self.rebuild_every = max(1, int(rebuild_every))
        self.adapt_enabled = bool(adapt)
        self.on_boundary = on_boundary
        self.terrain = terrain
        p = mesh.params
        self.wind_box = wind_box or (-0.5 * p["Lx"], 0.5 * p["Lx"], -0.5 * p["Ly"], 0.5 * p["Ly"])
        self.timings = dict(step=0.0, flag=0.0, forecast=0.0, layout=0.0, mesh=0.0,
                            transfer=0.0, capture=0.0)
        self.n_boundary = 0
        self.n_rebuild = 0
        self.steps = 0
        self.history = []          # (step, n_col, n_dof) after each rebuild
        self.log = []              # per boundary: step, vmax, plain split fraction, n_elem
        self._vmax = torch.zeros(1, dtype=torch.float64, device=q0.device)
        self._new_stepper(q0)
        self.q_prev = self.q.clone()

    # ------------------------------------------------------------------ #
    def _new_stepper(self, q):
        t0 = time.perf_counter()
        if self.lpc:
            api.sem_stage_tune(self.mesh, self.lpc)
        self.stepper = Stepper(self.mesh, q, self.dt, self.precision, graph=self.graph)
        torch.cuda.synchronize()
        self.timings["capture"] += time.perf_counter() - t0

    @property
    def q(self):
        return self.stepper.q

    def plain_flags(self):
        """The criterion's element and column flags (device int8)."""
        m = self.mesh
        ae = torch.empty(m.info["n_elem"], dtype=torch.int8, device="cuda")
        ac = torch.empty(m.info["n_col"], dtype=torch.int8, device="cuda")
        api.amr_flag(m, self.q, self.criterion, self.thresholds, self.lvl_max, ae, ac)
        return ae, ac

    def vmax(self):
        api.sem_max_wind(self.mesh, self.q, self.wind_box, self._vmax)
        return float(self._vmax.item())

    def boundary(self):
        """Diagnostics, the hook, and (every rebuild_every-th time) a rebuild.
        Returns True when the mesh changed."""
        t0 = time.perf_counter()
        k = self.n_boundary
        self.n_boundary += 1
        ae, ac = self.plain_flags()
        ae_h = ae.cpu().numpy()
        self.log.append(dict(step=self.steps, vmax=self.vmax(),
                             split_frac=float(np.mean(ae_h == 1)), n_elem=int(ae_h.size),
                             n_dof=int(self.mesh.n_dof)))
        self.timings["flag"] += time.perf_counter() - t0
        if self.on_boundary is not None:
            self.on_boundary(self, ae)
        changed = False
        if self.adapt_enabled and k % self.rebuild_every == 0:
            if self.forecaster is not None:
                t1 = time.perf_counter()
                ac = self.forecaster(self, ae, ac)
                torch.cuda.synchronize()
                self.timings["forecast"] += time.perf_counter() - t1
            changed = self._rebuild(ac.cpu().numpy())
        if not changed:
            self.q_prev = self.q.clone()
        return changed

    def _rebuild(self, flags):
        t1 = time.perf_counter()
        if not flags.any():
            return False
        cols = api.sem_adapt_columns(self.mesh, self.mesh.columns, flags, self.lvl_max)
        t2 = time.perf_counter()
        self.timings["layout"] += t2 - t1
        if _same_layout(cols, self.mesh.columns):
            return False
        new = self.mesh.with_columns(cols)
        new.set_reference(*self.reference)
        if self.terrain is not None:
            new.set_terrain(*self.terrain(new))
        T = api.Transfer(self.mesh, new)
        t3 = time.perf_counter()
        self.timings["mesh"] += t3 - t2
        q_new = new.state()
        api.sem_transfer_apply(T, self.q, q_new)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        self.timings["transfer"] += t4 - t3
        self.mesh = new
        self._new_stepper(q_new)
        self.q_prev = self.q.clone()
        self.n_rebuild += 1
        self.history.append((self.steps, int(new.info["n_col"]), int(new.n_dof)))
        return True

    # kept for callers that adapt by hand
    def adapt(self):
        return self.boundary()

    def run(self, n_steps):
        """Advance n_steps RK3 steps with a boundary every ``interval`` steps."""
        done = 0
        while done < n_steps:
            k = min(self.interval - (self.steps % self.interval), n_steps - done)
            t0 = time.perf_counter()
            self.stepper.step(k)
            torch.cuda.synchronize()
            self.timings["step"] += time.perf_counter() - t0
            done += k
            self.steps += k
            if self.steps % self.interval == 0:
                self.boundary()
        return self.q

    def wall(self):
        return sum(self.timings.values())
