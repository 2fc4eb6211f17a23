"""Hexahedral column mesh with hanging nodes (oracle, FP64).

Section 3 builds the solution from tensor-product LGL elements; Section 3.1
introduces hanging nodes on nonconforming faces; Section 4.1 refines only in
the horizontal, a whole column at a time (one hexahedron becomes a 2 x 2
block of hexahedra).  The mesh is therefore a horizontal quadtree of columns,
each column stacked over the same vertical layers.

This module derives everything geometrically from node coordinates, with no
use of the column structure beyond locating the columns that contain a point:

* unique global nodes: local nodes with equal (periodically wrapped)
  coordinates are one node, found by hashing rounded coordinates;
* a local node is *hanging* when it lies on the boundary of a coarser column
  without being one of that column's nodes (Section 3.1: the node has no
  counterpart on the coarse element); its value is the coarse element's
  polynomial evaluated there, and if that polynomial's nodes hang in turn
  the rows are composed until every source is a non-hanging node;
* Z (n_loc x n_dof, sparse): row l gives local node l as a combination of
  unique nodes (a unit row for a conforming node, Lagrange weights for a
  hanging one);
* lumped masses: m_L = w_i w_j w_k |J_e| and M_G = Z^T m_L (Section 3.1: the
  mass matrix is assembled through the same interpolation).

Local node order inside an element is l = i + (N+1)(j + (N+1)k) with i along
x, j along y, k along z (Section 3, basis definition).
"""

import numpy as np
import scipy.sparse as sp

from .gll import lgl_nodes, lgl_weights, lagrange_matrix


class OracleMesh:
    """Geometry, numbering, Z and masses of a column mesh.

    columns : int array (n_col, 3) of (level, ix, iy); column (l, ix, iy)
              covers [x_min + ix*Lx/(nx0*2^l), ...) with width Lx/(nx0*2^l);
              the domain is [-Lx/2, Lx/2] x [-Ly/2, Ly/2] x [z_0, z_nz].
    Element e = c * n_z + layer.
    """

    def __init__(self, N, nx0, ny0, Lx, Ly, z_edges, columns,
                 periodic_x=True, periodic_y=True):
        self.N = int(N)
        self.nx0, self.ny0 = int(nx0), int(ny0)
        self.Lx, self.Ly = float(Lx), float(Ly)
        self.z_edges = np.asarray(z_edges, dtype=np.float64)
        self.n_z = self.z_edges.size - 1
        self.columns = np.asarray(columns, dtype=np.int64).reshape(-1, 3)
        self.periodic_x, self.periodic_y = bool(periodic_x), bool(periodic_y)
        self.n_col = self.columns.shape[0]
        self.n_elem = self.n_col * self.n_z
        self.np1 = self.N + 1
        self.xi = lgl_nodes(self.N)
        self.w = lgl_weights(self.N)
        self._elements()
        self._numbering()

    # ------------------------------------------------------------------ #
    def _elements(self):
        N, n_z = self.N, self.n_z
        lev, ix, iy = self.columns.T
        wx = self.Lx / (self.nx0 * 2.0**lev)
        wy = self.Ly / (self.ny0 * 2.0**lev)
        x0 = -0.5 * self.Lx + ix * wx
        y0 = -0.5 * self.Ly + iy * wy
        self.col_wx, self.col_wy, self.col_x0, self.col_y0 = wx, wy, x0, y0
        rep = lambda a: np.repeat(a, n_z)
        self.e_level = rep(lev)
        self.e_col = np.repeat(np.arange(self.n_col), n_z)
        self.e_layer = np.tile(np.arange(n_z), self.n_col)
        self.e_x0, self.e_dx = rep(x0), rep(wx)
        self.e_y0, self.e_dy = rep(y0), rep(wy)
        self.e_z0 = self.z_edges[self.e_layer]
        self.e_dz = self.z_edges[self.e_layer + 1] - self.e_z0
        s = 0.5 * (1.0 + self.xi)
        E = self.n_elem
        n = self.np1
        # local coordinates, shape (E, k, j, i)
        self.xl = np.broadcast_to(
            (self.e_x0[:, None] + s[None, :] * self.e_dx[:, None])[:, None, None, :],
            (E, n, n, n)).copy()
        self.yl = np.broadcast_to(
            (self.e_y0[:, None] + s[None, :] * self.e_dy[:, None])[:, None, :, None],
            (E, n, n, n)).copy()
        self.zl = np.broadcast_to(
            (self.e_z0[:, None] + s[None, :] * self.e_dz[:, None])[:, :, None, None],
            (E, n, n, n)).copy()
        # lumped LGL mass per local node: w_i w_j w_k * dx dy dz / 8
        w3 = self.w[:, None, None] * self.w[None, :, None] * self.w[None, None, :]
        jac = self.e_dx * self.e_dy * self.e_dz / 8.0
        self.mL = (w3[None] * jac[:, None, None, None]).reshape(-1)

    def _wrap(self, x, L, periodic):
        if not periodic:
            return x
        x = np.where(x >= 0.5 * L - 1e-9 * L, x - L, x)
        return np.where(x < -0.5 * L - 1e-9 * L, x + L, x)

    def _keys(self, x, y, z):
        q = 1e-9 * max(self.Lx, self.Ly, self.z_edges[-1] - self.z_edges[0])
        xw = self._wrap(x, self.Lx, self.periodic_x)
        yw = self._wrap(y, self.Ly, self.periodic_y)
        return np.stack([np.rint(xw / q), np.rint(yw / q), np.rint(z / q)],
                        axis=-1).astype(np.int64)

    def _locate(self, level, xs, ys):
        """Columns of the given level whose closed box contains (xs, ys).

        Returns a list of (mask, column_id) candidate arrays (up to 4)."""
        nxl = self.nx0 * 2**level
        nyl = self.ny0 * 2**level
        grid = self._grids[level]
        wx, wy = self.Lx / nxl, self.Ly / nyl
        tx = (xs + 0.5 * self.Lx) / wx
        ty = (ys + 0.5 * self.Ly) / wy
        out = []
        for ax_t, nl, per in ((tx, nxl, self.periodic_x), (ty, nyl, self.periodic_y)):
            r = np.rint(ax_t)
            on = np.abs(ax_t - r) < 1e-9
            a = np.where(on, r, np.floor(ax_t)).astype(np.int64)
            b = np.where(on, r - 1, a).astype(np.int64)
            cand = []
            for c in (a, b):
                if per:
                    cand.append((np.ones_like(c, dtype=bool), np.mod(c, nl)))
                else:
                    ok = (c >= 0) & (c < nl)
                    cand.append((ok, np.clip(c, 0, nl - 1)))
            out.append(cand)
        res = []
        for okx, cx in out[0]:
            for oky, cy in out[1]:
                cid = grid[cx, cy]
                res.append((okx & oky & (cid >= 0), cid))
        return res

    def _numbering(self):
        N, n = self.N, self.np1
        E = self.n_elem
        lev = self.columns[:, 0]
        self.max_level = int(lev.max()) if self.n_col else 0
        self._grids = []
        for l in range(self.max_level + 1):
            g = -np.ones((self.nx0 * 2**l, self.ny0 * 2**l), dtype=np.int64)
            sel = np.nonzero(lev == l)[0]
            g[self.columns[sel, 1], self.columns[sel, 2]] = sel
            self._grids.append(g)
        X, Y, Zc = self.xl.reshape(-1), self.yl.reshape(-1), self.zl.reshape(-1)
        n_loc = X.size
        self.n_loc = n_loc
        e_of = np.repeat(np.arange(E), n**3)
        lvl_of = self.e_level[e_of]
        # --- hanging detection: coarser columns containing the point ------
        hang_col = -np.ones(n_loc, dtype=np.int64)
        for lc in range(self.max_level):
            cand = np.nonzero((lvl_of > lc) & (hang_col < 0))[0]
            if cand.size == 0:
                continue
            xs, ys = X[cand], Y[cand]
            for ok, cid in self._locate(lc, xs, ys):
                idx = np.nonzero(ok & (hang_col[cand] < 0))[0]
                if idx.size == 0:
                    continue
                c = cid[idx]
                dx = xs[idx] - self.col_x0[c]
                dy = ys[idx] - self.col_y0[c]
                if self.periodic_x:
                    dx = np.mod(dx + 1e-9 * self.Lx, self.Lx) - 1e-9 * self.Lx
                if self.periodic_y:
                    dy = np.mod(dy + 1e-9 * self.Ly, self.Ly) - 1e-9 * self.Ly
                sx = 2.0 * dx / self.col_wx[c] - 1.0
                sy = 2.0 * dy / self.col_wy[c] - 1.0
                isnode_x = np.min(np.abs(sx[:, None] - self.xi[None, :]), axis=1) < 1e-9
                isnode_y = np.min(np.abs(sy[:, None] - self.xi[None, :]), axis=1) < 1e-9
                hang = ~(isnode_x & isnode_y)
                hang_col[cand[idx[hang]]] = c[hang]
        self.hanging = hang_col >= 0
        # --- unique numbering of the non-hanging nodes --------------------
        keys = self._keys(X, Y, Zc)
        nh = np.nonzero(~self.hanging)[0]
        ukeys, first, inv = np.unique(keys[nh], axis=0, return_index=True,
                                      return_inverse=True)
        inv = inv.reshape(-1)
        self.n_dof = ukeys.shape[0]
        if self.hanging.any():
            # a hanging point may not also be a conforming node elsewhere;
            # hanging points shared by two fine elements are collapsed first
            u_hk = np.unique(keys[self.hanging], axis=0)
            _, cnt = np.unique(np.concatenate([ukeys, u_hk]), axis=0, return_counts=True)
            if np.any(cnt > 1):
                raise ValueError("a hanging point coincides with a conforming node "
                                 "(mesh violates 2:1 balance)")
        self.n_hang_points = int(np.unique(keys[self.hanging], axis=0).shape[0]) \
            if self.hanging.any() else 0
        self.node_xyz = np.stack([X[nh][first], Y[nh][first], Zc[nh][first]], axis=1)
        self.node_xyz[:, 0] = self._wrap(self.node_xyz[:, 0], self.Lx, self.periodic_x)
        self.node_xyz[:, 1] = self._wrap(self.node_xyz[:, 1], self.Ly, self.periodic_y)
        # --- Z: unit rows for conforming nodes ------------------------------
        Zm = sp.csr_matrix((np.ones(nh.size), (nh, inv)), shape=(n_loc, self.n_dof))
        # --- hanging rows, coarsest level first so sources are complete ----
        k_of = (np.arange(n_loc) // (n * n)) % n
        for l in range(1, self.max_level + 1):
            hs = np.nonzero(self.hanging & (lvl_of == l))[0]
            if hs.size == 0:
                continue
            c = hang_col[hs]
            dx = X[hs] - self.col_x0[c]
            dy = Y[hs] - self.col_y0[c]
            if self.periodic_x:
                dx = np.mod(dx + 1e-9 * self.Lx, self.Lx) - 1e-9 * self.Lx
            if self.periodic_y:
                dy = np.mod(dy + 1e-9 * self.Ly, self.Ly) - 1e-9 * self.Ly
            sx = 2.0 * dx / self.col_wx[c] - 1.0
            sy = 2.0 * dy / self.col_wy[c] - 1.0
            layer = self.e_layer[e_of[hs]]
            ec = c * self.n_z + layer                 # coarse element, same layer
            sz = 2.0 * (Zc[hs] - self.e_z0[ec]) / self.e_dz[ec] - 1.0
            Lx_ = lagrange_matrix(self.xi, sx)       # (nh, n)
            Ly_ = lagrange_matrix(self.xi, sy)
            Lz_ = lagrange_matrix(self.xi, sz)
            Wt = (Lz_[:, :, None, None] * Ly_[:, None, :, None] * Lx_[:, None, None, :])
            Wt = Wt.reshape(hs.size, n**3)
            src = ec[:, None] * n**3 + np.arange(n**3)[None, :]
            keep = np.abs(Wt) > 0.0
            rows = np.repeat(np.arange(hs.size), n**3).reshape(hs.size, n**3)[keep]
            W = sp.csr_matrix((Wt[keep], (rows, src[keep])), shape=(hs.size, n_loc))
            R = (W @ Zm).tocoo()
            Zm = Zm + sp.csr_matrix((R.data, (hs[R.row], R.col)), shape=(n_loc, self.n_dof))
        Zm.eliminate_zeros()
        self.Z = Zm.tocsr()
        self.ZT = self.Z.T.tocsr()
        self.MG = self.ZT @ self.mL
        H0, H1 = self.z_edges[0], self.z_edges[-1]
        tolz = 1e-9 * (H1 - H0)
        self.lid = (np.abs(self.node_xyz[:, 2] - H0) < tolz) | (np.abs(self.node_xyz[:, 2] - H1) < tolz)
        self.hanging_local = np.nonzero(self.hanging)[0]

    # ------------------------------------------------------------------ #
    def local_shape(self):
        return (self.n_elem, self.np1, self.np1, self.np1)

    def unique_keys(self, xyz):
        """Hash keys of arbitrary points (for matching numberings)."""
        return self._keys(xyz[:, 0], xyz[:, 1], xyz[:, 2])
