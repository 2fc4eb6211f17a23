"""Explicit third-order Runge-Kutta stages (FP64).

Section 5 integrates in time with an explicit third-order Runge-Kutta scheme
at constant time step without naming the variant.  The oracle takes the
strong-stability-preserving three-stage scheme of Shu and Osher in its
convex-combination form, one stage at a time:

    stage 1: q1   = q^n + dt R(q^n)
    stage 2: q2   = 3/4 q^n + 1/4 (q1 + dt R(q1))
    stage 3: q^{n+1} = 1/3 q^n + 2/3 (q2 + dt R(q2))

Each stage is q_out = a q^n + b q_s + c R(q_s) with (a, b, c) from
``stage_coefficients``.  A run of S stages repeats the pattern; after a
third stage, q^n is replaced by the stage output.
"""

import numpy as np


def stage_coefficients(s, dt):
    """(a, b, c) of stage s in {0, 1, 2}."""
    if s == 0:
        return 0.0, 1.0, dt
    if s == 1:
        return 0.75, 0.25, 0.25 * dt
    if s == 2:
        return 1.0 / 3.0, 2.0 / 3.0, (2.0 / 3.0) * dt
    raise ValueError("stage index must be 0, 1 or 2")


def stage_update(a, b, c, qn, qs, R):
    """q_out = a q^n + b q_s + c R."""
    return a * qn + b * qs + c * R


def run_stages(rhs_fn, q0, dt, n_stages):
    """Apply n_stages consecutive stages starting from q0 = q^n."""
    qn = np.array(q0, dtype=np.result_type(np.asarray(q0).dtype, np.float64), copy=True)
    qs = qn.copy()
    for st in range(n_stages):
        s = st % 3
        a, b, c = stage_coefficients(s, dt)
        qs = stage_update(a, b, c, qn, qs, rhs_fn(qs))
        if s == 2:
            qn = qs.copy()
    return qs, qn
