"""Python binding of the C ABI (argument marshalling only).

Every compute call forwards device pointers of contiguous torch tensors and
the current HIP stream to ``libsem.so``; no arithmetic of the method happens
here.  Function names match the C entry points.
"""

import ctypes

import numpy as np
import torch

from . import native
from .native import (SEM_FP64, SEM_FP32, SEM_SCATTER, SEM_GATHER, SEM_ASSEMBLE,  # noqa: F401
                     SEM_FINALIZE, SEM_CRIT_SPEED, SEM_CRIT_VORTZ)

NF = 5


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t, dtype, numel, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _desc(N, nx0, ny0, columns, Lx, Ly, z_edges, periodic_x, periodic_y, f, g, R_d, c_p, p00):
    cols = np.ascontiguousarray(np.asarray(columns, dtype=np.int32).reshape(-1, 3))
    lev = np.ascontiguousarray(cols[:, 0])
    ix = np.ascontiguousarray(cols[:, 1])
    iy = np.ascontiguousarray(cols[:, 2])
    z = np.ascontiguousarray(np.asarray(z_edges, dtype=np.float64))
    i32 = lambda a: a.ctypes.data_as(native.c_i32p)
    d = native.SemMeshDesc(int(N), int(nx0), int(ny0), int(z.size - 1), int(cols.shape[0]),
                           i32(lev), i32(ix), i32(iy), float(Lx), float(Ly),
                           z.ctypes.data_as(native.c_dp), int(bool(periodic_x)),
                           int(bool(periodic_y)), float(f), float(g), float(R_d), float(c_p),
                           float(p00))
    return (cols, lev, ix, iy, z), d


def _case_args(case):
    p = case["phys"]
    return (case["N"], case["nx0"], case["ny0"], case["columns"], case["Lx"], case["Ly"],
            case["z_edges"], case["periodic_x"], case["periodic_y"], p["f"], p["g"],
            p["R_d"], p["c_p"], p["p00"])


def sem_mesh_plan(case):
    """Host-only layout check and numbering (no GPU): returns
    (info dict, hxy, hhxy, z, mass) with mass the assembled M_G per unique node."""
    keep, d = _desc(*_case_args(case))
    info = native.SemMeshInfo()
    native.call("sem_mesh_plan", ctypes.byref(d), ctypes.byref(info), None, None, None, None)
    hxy = np.zeros((info.n_h, 2))
    hhxy = np.zeros((max(info.n_hh, 1), 2))
    z = np.zeros(info.nzn)
    mass = np.zeros(info.n_dof)
    dp = lambda a: a.ctypes.data_as(native.c_dp)
    native.call("sem_mesh_plan", ctypes.byref(d), ctypes.byref(info), dp(hxy), dp(hhxy), dp(z),
                dp(mass))
    out = {k: getattr(info, k) for k, _ in native.SemMeshInfo._fields_}
    return out, hxy, hhxy[: info.n_hh], z, mass


class Mesh:
    """Owns a ``sem_mesh`` handle built from a column layout."""

    def __init__(self, N, nx0, ny0, columns, Lx, Ly, z_edges, periodic_x=True,
                 periodic_y=True, f=0.0, g=9.81, R_d=287.0, c_p=1004.0, p00=1.0e5):
        self.params = dict(N=N, nx0=nx0, ny0=ny0, Lx=Lx, Ly=Ly, z_edges=z_edges,
                           periodic_x=periodic_x, periodic_y=periodic_y, f=f, g=g, R_d=R_d,
                           c_p=c_p, p00=p00)
        self._keep, d = _desc(N, nx0, ny0, columns, Lx, Ly, z_edges, periodic_x, periodic_y,
                              f, g, R_d, c_p, p00)
        self._d = d
        cols = self._keep[0]
        h = ctypes.c_void_p()
        native.call("sem_mesh_create", ctypes.byref(d), ctypes.byref(h))
        self.handle = h
        info = native.SemMeshInfo()
        native.call("sem_mesh_get_info", self.handle, ctypes.byref(info))
        self.info = {k: getattr(info, k) for k, _ in native.SemMeshInfo._fields_}
        self.columns = cols
        self.N = int(N)
        self.terrain = None

    @classmethod
    def from_case(cls, case):
        return cls(*_case_args(case))

    def with_columns(self, columns):
        """A new mesh with the same order, domain, vertical layers, physical
        constants and dissipation settings over another column layout."""
        new = Mesh(columns=columns, **self.params)
        if getattr(self, "dissipation", None):
            new.set_dissipation(*self.dissipation)
        return new

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                native.lib().sem_mesh_destroy(h)
            except Exception:
                pass
            self.handle = None

    # sizes
    @property
    def n_dof(self):
        return self.info["n_dof"]

    @property
    def n_hang(self):
        return self.info["n_hang"]

    @property
    def ldz(self):
        return self.info["ldz"]

    @property
    def n_state(self):
        """Doubles of a state array q[5][n_h][ldz] (padded rows)."""
        return NF * self.info["n_h"] * self.info["ldz"]

    @property
    def n_hstate(self):
        """Doubles of a hanging-point array hv[5][n_hh][ldz]."""
        return NF * self.info["n_hh"] * self.info["ldz"]

    def unpack(self, packed, device="cuda"):
        """Packed values (5, n_h*nzn) in [h][kz] order -> padded state tensor."""
        i = self.info
        a = torch.as_tensor(np.asarray(packed, dtype=np.float64)).reshape(NF, i["n_h"], i["nzn"])
        out = torch.zeros(NF, i["n_h"], i["ldz"], dtype=torch.float64)
        out[:, :, : i["nzn"]] = a
        return out.reshape(-1).to(device)

    def pack(self, state):
        """Padded state tensor -> numpy (5, n_h*nzn) in [h][kz] order."""
        i = self.info
        a = state.detach().reshape(NF, i["n_h"], i["ldz"])[:, :, : i["nzn"]]
        return a.cpu().numpy().reshape(NF, -1)

    def pack_hang(self, hv):
        i = self.info
        a = hv.detach().reshape(NF, i["n_hh"], i["ldz"])[:, :, : i["nzn"]]
        return a.cpu().numpy().reshape(NF, -1)

    @property
    def n_local(self):
        return self.info["n_local"]

    def coords(self):
        """(hxy (n_h,2), hhxy (n_hh,2), z (nzn,)) as numpy arrays."""
        i = self.info
        hxy = np.zeros((i["n_h"], 2))
        hhxy = np.zeros((max(i["n_hh"], 1), 2))
        z = np.zeros(i["nzn"])
        native.call("sem_mesh_coords", self.handle, hxy.ctypes.data_as(native.c_dp),
                    hhxy.ctypes.data_as(native.c_dp), z.ctypes.data_as(native.c_dp))
        return hxy, hhxy[: i["n_hh"]], z

    def node_xyz(self):
        """Coordinates of the unique nodes in state order [h][kz]."""
        hxy, _, z = self.coords()
        nzn = z.size
        out = np.empty((hxy.shape[0] * nzn, 3))
        out[:, 0] = np.repeat(hxy[:, 0], nzn)
        out[:, 1] = np.repeat(hxy[:, 1], nzn)
        out[:, 2] = np.tile(z, hxy.shape[0])
        return out

    def hang_xyz(self):
        _, hh, z = self.coords()
        nzn = z.size
        out = np.empty((hh.shape[0] * nzn, 3))
        out[:, 0] = np.repeat(hh[:, 0], nzn)
        out[:, 1] = np.repeat(hh[:, 1], nzn)
        out[:, 2] = np.tile(z, hh.shape[0])
        return out

    def set_reference(self, rho0, theta0, dtheta0dz):
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (rho0, theta0, dtheta0dz)]
        for a in arrs:
            if a.size != self.info["nzn"]:
                raise ValueError("reference arrays need one value per vertical node")
        native.call("sem_mesh_set_reference", self.handle,
                    *[a.ctypes.data_as(native.c_dp) for a in arrs])

    def set_dissipation(self, Cs=0.0, sponge_gamma=0.0, sponge_depth=4000.0):
        """Enable (or, with zeros, disable) the horizontal Smagorinsky-Lilly
        and absorbing-layer terms; see sem_mesh_set_dissipation."""
        native.call("sem_mesh_set_dissipation", self.handle, float(Cs), float(sponge_gamma),
                    float(sponge_depth))
        on = Cs > 0.0 or sponge_gamma > 0.0
        self.dissipation = (float(Cs), float(sponge_gamma), float(sponge_depth)) if on else None

    def set_terrain(self, zs, rho0=None, theta0=None, dtheta0dz=None):
        """Terrain-following coordinates (see sem_mesh_set_terrain): zs per
        unique horizontal node (coords() order), the reference state per unique
        node in state order [h][kz] at each node's physical height.  zs=None
        removes the terrain."""
        if zs is None:
            native.call("sem_mesh_set_terrain", self.handle, None, None, None, None)
            self.terrain = None
            return
        z = np.ascontiguousarray(np.asarray(zs, dtype=np.float64))
        if z.size != self.info["n_h"]:
            raise ValueError("zs needs one value per unique horizontal node")
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (rho0, theta0, dtheta0dz)]
        for a in arrs:
            if a.size != self.n_dof:
                raise ValueError("terrain reference arrays need one value per unique node")
        native.call("sem_mesh_set_terrain", self.handle, z.ctypes.data_as(native.c_dp),
                    *[a.ctypes.data_as(native.c_dp) for a in arrs])
        self.terrain = z.copy()

    def heights(self, zs=None):
        """Physical height of every unique node in state order, from the
        library (sem_mesh_heights): under the surface ``zs`` per unique
        horizontal node if given, else under the mesh's terrain (flat heights
        when none is set)."""
        out = np.zeros(self.n_dof)
        z = None
        if zs is not None:
            z = np.ascontiguousarray(np.asarray(zs, dtype=np.float64))
            if z.size != self.info["n_h"]:
                raise ValueError("zs needs one value per unique horizontal node")
        native.call("sem_mesh_heights", self.handle,
                    None if z is None else z.ctypes.data_as(native.c_dp),
                    out.ctypes.data_as(native.c_dp))
        return out

    def epoch(self):
        """Set-up epoch (sem_mesh_get_epoch): changes whenever a captured HIP
        graph of this mesh's compute calls would go stale."""
        e = ctypes.c_int64()
        native.call("sem_mesh_get_epoch", self.handle, ctypes.byref(e))
        return e.value

    def state(self, device="cuda"):
        """A zeroed state tensor (padding stays zero under every compute call)."""
        return torch.zeros(self.n_state, dtype=torch.float64, device=device)


def sem_nc_project(mesh, direction, src, dst, stream=None):
    nd, nh = mesh.n_state, mesh.n_hstate
    if direction == SEM_SCATTER:
        s, d = _ptr(src, torch.float64, nd, "src"), _ptr(dst, torch.float64, nh, "dst")
    else:
        s, d = _ptr(src, torch.float64, nh, "src"), _ptr(dst, torch.float64, nd, "dst")
    native.call("sem_nc_project", mesh.handle, int(direction), s, d, _stream(stream))


def sem_rhs(mesh, q, hv, rE, precision=SEM_FP64, stream=None):
    native.call("sem_rhs", mesh.handle, _ptr(q, torch.float64, mesh.n_state, "q"),
                _ptr(hv, torch.float64, mesh.n_hstate, "hv") if mesh.n_hang else None,
                _ptr(rE, torch.float64, NF * mesh.n_local, "rE"), int(precision), _stream(stream))


def sem_dss(mesh, phase, rE=None, acc=None, c=None, r=None, stream=None):
    native.call("sem_dss", mesh.handle, int(phase),
                _ptr(rE, torch.float64, NF * mesh.n_local, "rE"),
                _ptr(acc, torch.float64, mesh.n_state, "acc"),
                _ptr(c, torch.float64, mesh.n_hstate, "c") if mesh.n_hang else None,
                _ptr(r, torch.float64, mesh.n_state, "r"), _stream(stream))


def sem_stage_update(mesh, a, b, c, qn, qs, r, qout, stream=None):
    n = mesh.n_state
    native.call("sem_stage_update", mesh.handle, float(a), float(b), float(c),
                _ptr(qn, torch.float64, n, "qn"), _ptr(qs, torch.float64, n, "qs"),
                _ptr(r, torch.float64, n, "r"), _ptr(qout, torch.float64, n, "qout"),
                _stream(stream))


def sem_stage(mesh, a, b, c, qn, qs, qout, precision=SEM_FP64, stream=None):
    n = mesh.n_state
    native.call("sem_stage", mesh.handle, float(a), float(b), float(c),
                _ptr(qn, torch.float64, n, "qn"), _ptr(qs, torch.float64, n, "qs"),
                _ptr(qout, torch.float64, n, "qout"), int(precision), _stream(stream))


def amr_flag(mesh, q, criterion, thresholds, lvl_max, adapt_elem, adapt_col, stream=None):
    thr = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float64))
    if thr.size < lvl_max:
        raise ValueError("need one threshold per level")
    native.call("amr_flag", mesh.handle, _ptr(q, torch.float64, mesh.n_state, "q"),
                int(criterion), thr.ctypes.data_as(native.c_dp) if thr.size else None,
                int(lvl_max), _ptr(adapt_elem, torch.int8, mesh.info["n_elem"], "adapt_elem"),
                _ptr(adapt_col, torch.int8, mesh.info["n_col"], "adapt_col"), _stream(stream))


def sem_stage_tune(mesh, layers_per_chunk=0):
    native.call("sem_stage_tune", mesh.handle, int(layers_per_chunk))


def sem_stage_get_tune(mesh):
    a = ctypes.c_int()
    native.call("sem_stage_get_tune", mesh.handle, ctypes.byref(a))
    return a.value


SEM_LAYOUT_COLUMNS, SEM_LAYOUT_BLOCKS, SEM_LAYOUT_COLUMNS_KZ, SEM_LAYOUT_COLUMNS_SPLIT = 0, 1, 2, 3


def sem_stage_set_layout(mesh, layout, param=0):
    native.call("sem_stage_set_layout", mesh.handle, int(layout), int(param))


def sem_stage_get_layout(mesh):
    """(layout, param): layers per chunk of the column layout, or the number
    of vertical segments of the block layout."""
    lay, par = ctypes.c_int(), ctypes.c_int()
    native.call("sem_stage_get_layout", mesh.handle, ctypes.byref(lay), ctypes.byref(par))
    return lay.value, par.value


def sem_stage_autotune(mesh, qn, qs, qout, precision=SEM_FP64, reps=5, stream=None):
    """Pick the fastest chunk depth on this mesh; returns (layers_per_chunk, ms)."""
    n = mesh.n_state
    lpc, ms = ctypes.c_int(), ctypes.c_float()
    native.call("sem_stage_autotune", mesh.handle, _ptr(qn, torch.float64, n, "qn"),
                _ptr(qs, torch.float64, n, "qs"), _ptr(qout, torch.float64, n, "qout"),
                int(precision), int(reps), ctypes.byref(lpc), ctypes.byref(ms), _stream(stream))
    return lpc.value, ms.value


def _desc_of(params, columns):
    p = params
    return _desc(p["N"], p["nx0"], p["ny0"], columns, p["Lx"], p["Ly"], p["z_edges"],
                 p["periodic_x"], p["periodic_y"], p["f"], p["g"], p["R_d"], p["c_p"], p["p00"])


def sem_adapt_columns(mesh_or_params, columns, adapt_col, lvl_max):
    """One adaptation pass of a column layout (host only).  ``mesh_or_params``
    is a Mesh or its ``params`` dict; ``adapt_col`` holds one flag per column
    (numpy or a torch tensor).  Returns the new layout (n, 3) int32."""
    params = mesh_or_params.params if isinstance(mesh_or_params, Mesh) else mesh_or_params
    keep, d = _desc_of(params, columns)
    if isinstance(adapt_col, torch.Tensor):
        adapt_col = adapt_col.detach().cpu().numpy()
    fl = np.ascontiguousarray(np.asarray(adapt_col, dtype=np.int8).reshape(-1))
    if fl.size != keep[0].shape[0]:
        raise ValueError("one flag per column")
    n = ctypes.c_int32()
    L = native.lib()
    i32 = lambda a: a.ctypes.data_as(native.c_i32p)
    # room for every column split once (the usual case); the call reports the
    # size needed when that is not enough, and runs again with it
    cap = 4 * fl.size + 1024
    for _ in range(2):
        lev, ix, iy = (np.zeros(cap, np.int32) for _ in range(3))
        rc = L.sem_adapt_columns(ctypes.byref(d), fl.ctypes.data_as(ctypes.c_void_p), int(lvl_max), cap,
                                 i32(lev), i32(ix), i32(iy), ctypes.byref(n))
        if rc == native.SEM_OK:
            k = n.value
            return np.stack([lev[:k], ix[:k], iy[:k]], axis=1)
        if n.value <= cap:
            raise native.SemError("sem_adapt_columns", rc, L.sem_last_error().decode())
        cap = n.value
    raise native.SemError("sem_adapt_columns", rc, L.sem_last_error().decode())


def sem_transfer_plan(params, columns_from, columns_to):
    """Host-only transfer rows (ptr, src, w) from one layout to another."""
    ka, da = _desc_of(params, columns_from)
    kb, db = _desc_of(params, columns_to)
    nnz = ctypes.c_int64()
    native.call("sem_transfer_plan", ctypes.byref(da), ctypes.byref(db), ctypes.byref(nnz),
                None, None, None)
    info = native.SemMeshInfo()
    native.call("sem_mesh_plan", ctypes.byref(db), ctypes.byref(info), None, None, None, None)
    ptr = np.zeros(info.n_h + 1, np.int32)
    src = np.zeros(max(nnz.value, 1), np.int32)
    w = np.zeros(max(nnz.value, 1))
    native.call("sem_transfer_plan", ctypes.byref(da), ctypes.byref(db), ctypes.byref(nnz),
                ptr.ctypes.data_as(native.c_i32p), src.ctypes.data_as(native.c_i32p),
                w.ctypes.data_as(native.c_dp))
    return ptr, src[: nnz.value], w[: nnz.value]


class Transfer:
    """Owns a ``sem_transfer`` handle from mesh ``src`` to mesh ``dst``."""

    def __init__(self, src, dst):
        h = ctypes.c_void_p()
        native.call("sem_transfer_create", src.handle, dst.handle, ctypes.byref(h))
        self.handle = h
        self.n_from, self.n_to = src.n_state, dst.n_state

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                native.lib().sem_transfer_destroy(h)
            except Exception:
                pass
            self.handle = None


def sem_transfer_apply(transfer, q_from, q_to, stream=None):
    native.call("sem_transfer_apply", transfer.handle,
                _ptr(q_from, torch.float64, transfer.n_from, "q_from"),
                _ptr(q_to, torch.float64, transfer.n_to, "q_to"), _stream(stream))


# ---------------------------------------------------------------- forecaster
NFEAT = native.SEM_NFEAT
MLP_NPARAM = native.SEM_MLP_NPARAM
MLP_WORK = native.SEM_MLP_WORK


def amr_features(mesh, q, q_prev, plain_elem, criterion, thresholds, lvl_max, scale, feat, dem,
                 stream=None):
    thr = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float64))
    if thr.size < lvl_max:
        raise ValueError("need one threshold per level")
    sc = np.ascontiguousarray(np.asarray(scale, dtype=np.float32))
    if sc.size != NFEAT:
        raise ValueError("one scale per feature")
    ne = mesh.info["n_elem"]
    native.call("amr_features", mesh.handle, _ptr(q, torch.float64, mesh.n_state, "q"),
                _ptr(q_prev, torch.float64, mesh.n_state, "q_prev"),
                _ptr(plain_elem, torch.int8, ne, "plain_elem"), int(criterion),
                thr.ctypes.data_as(native.c_dp) if thr.size else None, int(lvl_max),
                sc.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                _ptr(feat, torch.float32, ne * NFEAT, "feat"), _ptr(dem, torch.int8, ne, "dem"),
                _stream(stream))


def amr_forecast_flags(mesh, logits, plain_elem, lvl_max, adapt_elem, adapt_col, stream=None):
    ne = mesh.info["n_elem"]
    native.call("amr_forecast_flags", mesh.handle, _ptr(logits, torch.float32, 3 * ne, "logits"),
                _ptr(plain_elem, torch.int8, ne, "plain_elem"), int(lvl_max),
                _ptr(adapt_elem, torch.int8, ne, "adapt_elem"),
                _ptr(adapt_col, torch.int8, mesh.info["n_col"], "adapt_col"), _stream(stream))


def sem_max_wind(mesh, q, box, out, stream=None):
    """out (1-element float64 CUDA tensor) = max horizontal wind in box
    (x0, x1, y0, y1)."""
    x0, x1, y0, y1 = (float(b) for b in box)
    native.call("sem_max_wind", mesh.handle, _ptr(q, torch.float64, mesh.n_state, "q"), x0, x1,
                y0, y1, _ptr(out, torch.float64, 1, "out"), _stream(stream))


def sem_forecast_labels(params, columns_at, columns_later, dem_later):
    """Host-only training classes (n_elem(at),) int8 in {0, 1, 2}."""
    ka, da = _desc_of(params, columns_at)
    kb, db = _desc_of(params, columns_later)
    nz = len(params["z_edges"]) - 1
    dem = np.ascontiguousarray(np.asarray(dem_later, dtype=np.int8).reshape(-1))
    if dem.size != kb[0].shape[0] * nz:
        raise ValueError("one dem value per element of the later layout")
    out = np.zeros(ka[0].shape[0] * nz, dtype=np.int8)
    native.call("sem_forecast_labels", ctypes.byref(da), ctypes.byref(db),
                dem.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p))
    return out


def mlp_forward(params, x, logits, stream=None):
    n = x.shape[0]
    native.call("mlp_forward", _ptr(params, torch.float32, MLP_NPARAM, "params"),
                _ptr(x, torch.float32, n * 16, "x"), int(n),
                _ptr(logits, torch.float32, n * 3, "logits"), _stream(stream))


def mlp_backward(params, x, cls, idx, work, grad, loss, stream=None):
    """Gradient of the mean cross-entropy over the rows idx (or all rows)."""
    rows = x.shape[0]
    n = rows if idx is None else idx.numel()
    if work.numel() < n * MLP_WORK:
        raise ValueError("workspace too small")
    native.call("mlp_backward", _ptr(params, torch.float32, MLP_NPARAM, "params"),
                _ptr(x, torch.float32, rows * 16, "x"), int(rows),
                _ptr(cls, torch.int8, rows, "cls"),
                None if idx is None else _ptr(idx, torch.int32, n, "idx"), int(n),
                _ptr(work, torch.float32, work.numel(), "work"),
                _ptr(grad, torch.float32, MLP_NPARAM, "grad"), _ptr(loss, torch.float32, 1, "loss"),
                _stream(stream))


def mlp_backward_noalloc(params, x, cls, idx, grad, loss, stream=None):
    """mlp_backward with the library's own per-GPU workspace (no caller
    allocation); at most SEM_MLP_NOALLOC_MAX samples per call."""
    rows = x.shape[0]
    n = rows if idx is None else idx.numel()
    native.call("mlp_backward_noalloc", _ptr(params, torch.float32, MLP_NPARAM, "params"),
                _ptr(x, torch.float32, rows * 16, "x"), int(rows),
                _ptr(cls, torch.int8, rows, "cls"),
                None if idx is None else _ptr(idx, torch.int32, n, "idx"), int(n),
                _ptr(grad, torch.float32, MLP_NPARAM, "grad"), _ptr(loss, torch.float32, 1, "loss"),
                _stream(stream))


def mlp_adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    native.call("mlp_adam_step", _ptr(params, torch.float32, MLP_NPARAM, "params"),
                _ptr(grad, torch.float32, MLP_NPARAM, "grad"), _ptr(m, torch.float32, MLP_NPARAM, "m"),
                _ptr(v, torch.float32, MLP_NPARAM, "v"), int(t), float(lr), float(beta1),
                float(beta2), float(eps), _stream(stream))
