"""Dynamic h-adaptation driver (Section 4.1 and Algorithm 1 of the paper:
evaluate the refinement criterion, adapt the column quadtree, move the
solution, continue stepping).

Every ``interval`` RK3 steps ``AdaptiveRun.adapt`` does, on the device unless
noted:

1. ``amr_flag`` -> per-column flags (+1 split, -1 merge, 0 keep);
2. optionally, a forecaster (a callable taking the run and the criterion's
   element and column flags and returning combined column flags on the
   device);
3. ``sem_adapt_columns`` (host) -> the new layout (split, 2:1 balance,
   merge);
4. a new mesh handle over the new layout, its reference state (the vertical
   structure is unchanged, so the same per-level arrays are reused), the
   transfer rows, one ``sem_transfer_apply`` launch;
5. a new ``Stepper`` (HIP graphs recaptured for the new mesh).

The wall time of each phase is accumulated in ``timings``.
"""

import time

import numpy as np
import torch

from . import api
from .solver import Stepper


class AdaptiveRun:
    def __init__(self, mesh, q0, dt, reference, criterion, thresholds, lvl_max,
                 interval, precision=api.SEM_FP64, graph=True, layers_per_chunk=0,
                 forecaster=None):
        """mesh: api.Mesh; q0: padded state tensor on it; reference: tuple of
        (rho0, theta0, dtheta0dz) per vertical node (already set on mesh)."""
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
        self.timings = dict(step=0.0, flag=0.0, layout=0.0, mesh=0.0, transfer=0.0, capture=0.0)
        self.n_adapt = 0
        self.n_rebuild = 0
        self.steps = 0
        self.history = []          # (step, n_col, n_dof) after each rebuild
        self._new_stepper(q0)

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

    def flags(self):
        """Per-column flags of the plain criterion (device int8) and, when a
        forecaster is attached, the combined flags."""
        m = self.mesh
        ae = torch.empty(m.info["n_elem"], dtype=torch.int8, device="cuda")
        ac = torch.empty(m.info["n_col"], dtype=torch.int8, device="cuda")
        api.amr_flag(m, self.q, self.criterion, self.thresholds, self.lvl_max, ae, ac)
        if self.forecaster is not None:
            ac = self.forecaster(self, ae, ac)
        return ae, ac

    def adapt(self):
        """One adaptation pass; returns True when the mesh changed."""
        t0 = time.perf_counter()
        _, ac = self.flags()
        flags = ac.cpu().numpy()
        t1 = time.perf_counter()
        self.timings["flag"] += t1 - t0
        self.n_adapt += 1
        if not flags.any():
            return False
        cols = api.sem_adapt_columns(self.mesh, self.mesh.columns, flags, self.lvl_max)
        t2 = time.perf_counter()
        self.timings["layout"] += t2 - t1
        if len(cols) == len(self.mesh.columns) and \
                {tuple(c) for c in cols.tolist()} == {tuple(c) for c in self.mesh.columns.tolist()}:
            return False
        new = self.mesh.with_columns(cols)
        new.set_reference(*self.reference)
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
        self.n_rebuild += 1
        self.history.append((self.steps, int(new.info["n_col"]), int(new.n_dof)))
        return True

    def run(self, n_steps, adapt_first=False):
        """Advance n_steps RK3 steps, adapting every ``interval`` steps."""
        if adapt_first:
            self.adapt()
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
                self.adapt()
        return self.q

