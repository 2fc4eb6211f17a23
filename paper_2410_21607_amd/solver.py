"""Explicit SSP-RK3 time stepping on the fused stage (Section 5 of the paper:
explicit third-order Runge-Kutta at constant time step).

One time step is three calls of ``sem_stage``:

    q1      = sem_stage(a=0,   b=1,   c=dt;      q^n, q^n)
    q2      = sem_stage(a=3/4, b=1/4, c=dt/4;    q^n, q1)
    q^{n+1} = sem_stage(a=1/3, b=2/3, c=2 dt/3;  q^n, q2)

With ``graph=True`` the three launches (and every kernel inside them) are
captured once per buffer parity into HIP graphs and replayed; two graphs
alternate the roles of the two state buffers, so no copy is needed.  The
graphs remember the mesh's set-up epoch at capture; a replay after any call
that changed the mesh's tables or settings (re-tuning, terrain, dissipation)
captures them again first, so a stale graph is never replayed.
"""

import torch

from . import api

SSP_RK3 = ((0.0, 1.0, 1.0), (0.75, 0.25, 0.25), (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0))


def stage_coefficients(s, dt):
    a, b, c = SSP_RK3[s]
    return a, b, c * dt


class Stepper:
    """Owns the state buffers of one mesh and advances them in time."""

    def __init__(self, mesh, q0, dt, precision=api.SEM_FP64, graph=False):
        self.mesh = mesh
        self.dt = float(dt)
        self.precision = precision
        n = mesh.n_state
        if q0.numel() != n:
            raise ValueError("initial state has the wrong size (expected the padded layout)")
        # zero-filled so that the row padding stays zero (no call writes it)
        self.buf = [q0.detach().to(torch.float64).contiguous().clone(),
                    torch.zeros(n, dtype=torch.float64, device=q0.device)]
        self.s1 = torch.zeros(n, dtype=torch.float64, device=q0.device)
        self.s2 = torch.zeros(n, dtype=torch.float64, device=q0.device)
        self.cur = 0
        self.steps = 0
        self.graphs = None
        self.captures = 0
        self.epoch = None
        if graph:
            self._capture()

    @property
    def q(self):
        return self.buf[self.cur]

    def _step_eager(self, src, dst, stream=None):
        m, p, dt = self.mesh, self.precision, self.dt
        a, b, c = stage_coefficients(0, dt)
        api.sem_stage(m, a, b, c, src, src, self.s1, p, stream)
        a, b, c = stage_coefficients(1, dt)
        api.sem_stage(m, a, b, c, src, self.s1, self.s2, p, stream)
        a, b, c = stage_coefficients(2, dt)
        api.sem_stage(m, a, b, c, src, self.s2, dst, p, stream)

    def _capture(self):
        # warm the kernels up on a side stream, then capture both parities
        self.graphs = None
        self.epoch = self.mesh.epoch()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        save = [b.clone() for b in self.buf]
        with torch.cuda.stream(s):
            self._step_eager(self.buf[0], self.buf[1], s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        for b, v in zip(self.buf, save):
            b.copy_(v)
        self.graphs = []
        for parity in (0, 1):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                self._step_eager(self.buf[parity], self.buf[1 - parity],
                                 torch.cuda.current_stream())
            self.graphs.append(g)
        torch.cuda.synchronize()
        self.captures += 1

    def step(self, n=1):
        """Advance n full RK3 steps (3 stages each)."""
        for _ in range(n):
            if self.graphs is not None:
                if self.mesh.epoch() != self.epoch:
                    self._capture()
                self.graphs[self.cur].replay()
            else:
                self._step_eager(self.buf[self.cur], self.buf[1 - self.cur])
            self.cur = 1 - self.cur
            self.steps += 1
        return self.q
