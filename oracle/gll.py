"""Legendre-Gauss-Lobatto (LGL) basis in FP64.

Section 3 of the paper builds the element basis as tensor products of the
1-D Lagrange polynomials of order N through the LGL points, and uses the same
points for quadrature (inexact integration, lumped mass).  This module writes
out the textbook definitions of those objects:

* nodes   : -1, the N-1 roots of P_N'(xi), +1
* weights : w_i = 2 / (N (N+1) P_N(xi_i)^2)
* D       : D[i, j] = l_j'(xi_i) (derivative of the j-th Lagrange polynomial
            evaluated at node i)
* interp  : L[p, j] = l_j(s_p) for arbitrary points s_p
"""

import numpy as np
from numpy.polynomial import legendre as L


def lgl_nodes(N):
    """LGL nodes on [-1, 1]: endpoints plus the roots of P_N' (Section 3)."""
    if N < 1:
        raise ValueError("order N must be >= 1")
    if N == 1:
        return np.array([-1.0, 1.0])
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    dP = L.legder(cN)
    interior = np.sort(np.real(L.legroots(dP)))
    # polish the companion-matrix roots with Newton on P_N'
    d2P = L.legder(dP)
    for _ in range(6):
        interior = interior - L.legval(interior, dP) / L.legval(interior, d2P)
    x = np.concatenate(([-1.0], interior, [1.0]))
    # enforce exact symmetry x_i = -x_{N-i}
    x = 0.5 * (x - x[::-1])
    return x


def lgl_weights(N):
    """LGL quadrature weights w_i = 2 / (N (N+1) P_N(x_i)^2)."""
    x = lgl_nodes(N)
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    PN = L.legval(x, cN)
    return 2.0 / (N * (N + 1) * PN**2)


def lagrange_matrix(nodes, s):
    """L[p, j] = l_j(s_p): the product form of the Lagrange polynomials."""
    nodes = np.asarray(nodes, dtype=np.float64)
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    n = nodes.size
    out = np.ones((s.size, n))
    for j in range(n):
        for k in range(n):
            if k != j:
                out[:, j] *= (s - nodes[k]) / (nodes[j] - nodes[k])
    return out


def derivative_matrix(N):
    """D[i, j] = l_j'(x_i) from the derivative of the product form.

    l_j'(x) = sum_{m != j} 1/(x_j - x_m) prod_{k != j, m} (x - x_k)/(x_j - x_k)
    evaluated literally at every node.
    """
    x = lgl_nodes(N)
    n = N + 1
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for m in range(n):
                if m == j:
                    continue
                term = 1.0 / (x[j] - x[m])
                for k in range(n):
                    if k != j and k != m:
                        term *= (x[i] - x[k]) / (x[j] - x[k])
                acc += term
            D[i, j] = acc
    return D
