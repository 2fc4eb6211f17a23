"""Error norms and wind diagnostics used to compare two solutions.

* Floor-scaled relative L2 error per field over unique nodes:
  ||a - b||_2 / max(||b||_2, s_f sqrt(n)); the floor s_f keeps nearly-zero
  fields (w, the lid-adjacent tendencies) from making the ratio meaningless.
* Maximum horizontal wind inside a horizontal sub-box (Section 5.2 measures
  the maximum of sqrt(u^2 + v^2) inside [-50, 50] km x [-50, 50] km over the
  full depth).
"""

import numpy as np

# state floors (rho' kg/m3, u v w m/s, theta' K); tendency floors are these
# per 1000 s
STATE_FLOORS = np.array([1e-3, 1.0, 1.0, 1.0, 0.1])
RHS_FLOORS = STATE_FLOORS * 1e-3


def rel_l2(a, b, floors):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.empty(a.shape[0])
    for f in range(a.shape[0]):
        n = a[f].size
        den = max(np.linalg.norm(b[f]), floors[f] * np.sqrt(n))
        out[f] = np.linalg.norm(a[f] - b[f]) / den
    return out


def max_wind(xyz, q, half_width=50e3):
    """max sqrt(u^2+v^2) over nodes with |x|,|y| <= half_width."""
    sel = (np.abs(xyz[:, 0]) <= half_width) & (np.abs(xyz[:, 1]) <= half_width)
    if not sel.any():
        return 0.0
    return float(np.sqrt(q[1, sel] ** 2 + q[2, sel] ** 2).max())
