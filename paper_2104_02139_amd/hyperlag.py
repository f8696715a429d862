"""ctypes binding of libhyperlag.so (C-ABI in ``include/hyperlag.h``).

Argument marshalling only: every step of the method runs in the HIP
kernels of the library.  Arrays may be numpy arrays (host memory) or torch
tensors on the GPU (device memory, passed by ``data_ptr()``).  There is no
CPU fallback: if the library is missing or no GPU is present the calls
raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhyperlag.so")

HL_X, HL_VHAT, HL_TAU, HL_V, HL_E, HL_B, HL_VSTAR, HL_ORDER, HL_MASS, HL_T = range(10)
FIELDS = dict(x=HL_X, vhat=HL_VHAT, tau=HL_TAU, v=HL_V, e=HL_E, B=HL_B, vstar=HL_VSTAR,
              order=HL_ORDER, mass=HL_MASS, T=HL_T)

# every exported symbol of the C-ABI
EXPORTS = ["hl_create", "hl_destroy", "hl_mesh_upload", "hl_state_init", "hl_set_params",
           "hl_compute_dt", "hl_step", "hl_step_replay", "hl_query", "hl_upload_field",
           "hl_profile_enable", "hl_profile_reset", "hl_profile_get", "hl_status_str",
           "hl_last_error", "hl_mesh_upload_batch", "hl_step_batch", "hl_query_dt", "hl_use_graph",
           "hl_forward_record", "hl_forward_replay", "hl_adjoint_run", "hl_tape_get",
           "hl_set_schedule", "hl_get_schedule", "hl_autotune", "hl_set_boundary_loads",
           "hl_set_contact", "hl_get_contact", "hl_mesh_refine", "hl_mesh_info", "hl_mesh_get",
           "hl_set_numbering", "hl_mesh_check", "hl_state_save", "hl_state_restore",
           "hl_acoustic_dt_noalloc", "hl_group_create", "hl_group_destroy", "hl_group_use_graph",
           "hl_group_step", "hl_measure_peaks"]

# internal numbering of uploaded meshes (hl_set_numbering)
NUMBERING_KEEP, NUMBERING_SPATIAL = 0, 1
HL_OK, HL_E_INVALID, HL_E_DEGENERATE_CELL, HL_E_NONCONFORMING = 0, -1, -2, -3

# stages of the full-mesh part of a step (launch schedules)
STAGES = ("pack", "node_agg", "predict", "node_solve", "update")


class Params(C.Structure):
    _fields_ = [("c_cfl", C.c_double), ("c_v", C.c_double), ("c_i", C.c_double),
                ("delta0", C.c_double), ("delta1", C.c_double), ("eps_tol", C.c_double),
                ("detect", C.c_int32), ("cascade", C.c_int32), ("shear_a", C.c_double),
                ("eos", C.c_int32), ("reserved", C.c_int32), ("sg_gamma", C.c_double), ("sg_pinf", C.c_double)]


def default_params(dim=3, detect=True, c_cfl=None, cascade=2, shear_a=-1.0, eos=0, sg_gamma=2.2, sg_pinf=1e6):
    """Paper values (Sections 3.5, 3.6); cascade 2: P1 -> P0, 3: P1 -> P1
    with the Barth-Jespersen limiter -> P0; shear_a: shear energy family
    (-1 neo-Hookean, 0 the paper's non-linear law); eos 1: the stiffened
    gas with sg_gamma and sg_pinf."""
    return Params(c_cfl if c_cfl is not None else (0.4 if dim == 2 else 0.25),
                  0.2, 0.1, 1e-4, 1e-3, 1e-12, 1 if detect else 0, int(cascade), float(shear_a),
                  int(eos), 0, float(sg_gamma), float(sg_pinf))


class StepInfo(C.Structure):
    _fields_ = [("dt_used", C.c_double), ("dt_next", C.c_double), ("dt_acoustic", C.c_double),
                ("dt_volume", C.c_double), ("mass", C.c_double), ("mom", C.c_double * 3),
                ("energy", C.c_double), ("kinetic", C.c_double), ("elastic", C.c_double),
                ("n_p0", C.c_int64), ("n_flag_first", C.c_int64), ("mood_iters", C.c_int32),
                ("status", C.c_int32), ("n_limited", C.c_int64), ("n_contact", C.c_int64),
                ("trials", C.c_int32), ("clipped", C.c_int32), ("n_recomputed", C.c_int64),
                ("gcl_defect", C.c_double), ("detB_defect", C.c_double), ("n_detB", C.c_int64)]

    def as_dict(self):
        return dict(dt_used=self.dt_used, dt_next=self.dt_next, dt_acoustic=self.dt_acoustic,
                    dt_volume=self.dt_volume, mass=self.mass, mom=list(self.mom),
                    energy=self.energy, kinetic=self.kinetic, elastic=self.elastic,
                    n_p0=self.n_p0, n_flag_first=self.n_flag_first,
                    mood_iters=self.mood_iters, status=self.status, n_limited=self.n_limited,
                    n_contact=self.n_contact, trials=self.trials, clipped=self.clipped,
                    n_recomputed=self.n_recomputed, gcl_defect=self.gcl_defect,
                    detB_defect=self.detB_defect, n_detB=self.n_detB)


class Schedule(C.Structure):
    _fields_ = [("tile", C.c_int32), ("block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("reserved", C.c_int32)]


class HyperLagError(RuntimeError):
    pass


_lib = None


def load():
    """Load libhyperlag.so from the package directory (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HyperLagError(f"{LIB_PATH} is not built; run `python -m paper_2104_02139_amd.build`")
    # PyTorch ships its own HIP runtime.  Loading it first makes the
    # library bind to that same runtime (one runtime per process), so
    # torch's streams and device pointers are valid handles here and torch
    # can still initialise the GPU after the library has used it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i64, dp = C.c_void_p, C.c_int64, C.c_double
    L.hl_status_str.restype = C.c_char_p
    L.hl_status_str.argtypes = [C.c_int]
    L.hl_last_error.restype = C.c_char_p
    L.hl_last_error.argtypes = []
    L.hl_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    L.hl_destroy.argtypes = [vp]
    L.hl_mesh_upload.argtypes = [vp, C.c_int, i64, vp, i64, vp, vp, vp, C.c_int]
    L.hl_mesh_upload_batch.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, C.c_int]
    L.hl_step_batch.argtypes = [vp, vp, C.c_int, C.POINTER(StepInfo)]
    L.hl_query_dt.argtypes = [vp, vp, C.c_int, C.c_int]
    L.hl_use_graph.argtypes = [vp, C.c_int, C.c_int]
    L.hl_forward_record.argtypes = [vp, C.c_int, C.c_int]
    L.hl_forward_replay.argtypes = [vp]
    L.hl_adjoint_run.argtypes = [vp, vp, vp, vp, vp, C.c_int]
    L.hl_tape_get.argtypes = [vp, C.c_int, vp, vp]
    L.hl_state_init.argtypes = [vp, vp, vp, vp, vp, vp, C.POINTER(Params), C.c_int]
    L.hl_set_params.argtypes = [vp, C.POINTER(Params)]
    L.hl_set_boundary_loads.argtypes = [vp, i64, vp, vp, vp, vp, C.c_int]
    L.hl_set_contact.argtypes = [vp, i64, vp, vp, vp, C.c_int]
    L.hl_mesh_refine.argtypes = [vp, C.c_int]
    L.hl_mesh_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(i64), C.POINTER(i64)]
    L.hl_mesh_get.argtypes = [vp, vp, vp, vp, vp, C.c_int]
    L.hl_get_contact.argtypes = [vp, vp, i64]
    L.hl_compute_dt.argtypes = [vp, C.POINTER(dp)]
    L.hl_step.argtypes = [vp, dp, C.POINTER(StepInfo)]
    L.hl_step_replay.argtypes = [vp, dp, vp, C.c_int, C.POINTER(StepInfo)]
    L.hl_query.argtypes = [vp, C.c_int, vp, i64, C.c_int]
    L.hl_upload_field.argtypes = [vp, C.c_int, vp, i64, C.c_int]
    L.hl_set_schedule.argtypes = [vp, C.c_int, C.POINTER(Schedule)]
    L.hl_get_schedule.argtypes = [vp, C.c_int, C.POINTER(Schedule)]
    L.hl_autotune.argtypes = [vp, C.c_int, vp]
    L.hl_profile_enable.argtypes = [vp, C.c_int]
    L.hl_profile_reset.argtypes = [vp]
    L.hl_profile_get.argtypes = [vp, C.c_char_p, C.POINTER(dp), C.POINTER(i64)]
    L.hl_set_numbering.argtypes = [vp, C.c_int]
    L.hl_mesh_check.argtypes = [C.c_int, i64, vp, i64, vp]
    L.hl_state_save.argtypes = [vp, vp, C.POINTER(i64)]
    L.hl_state_restore.argtypes = [vp, vp, i64]
    L.hl_acoustic_dt_noalloc.argtypes = [C.c_int, vp, C.c_int, i64, vp, i64, vp, vp, vp, vp, vp, dp, vp]
    L.hl_group_create.argtypes = [C.POINTER(vp), vp, vp]
    L.hl_group_destroy.argtypes = [vp]
    L.hl_group_use_graph.argtypes = [vp, C.c_int, C.c_int]
    L.hl_group_step.argtypes = [vp, vp, vp]
    L.hl_measure_peaks.argtypes = [C.c_int, vp, i64, C.POINTER(dp), C.POINTER(dp)]
    for name in EXPORTS:
        if name not in ("hl_status_str", "hl_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc, what):
    if rc < 0:
        msg = load().hl_status_str(rc).decode()
        detail = load().hl_last_error().decode()
        # HIP errors carry their detail; so do an invalid group and an
        # adjoint request the recorded run does not support
        if rc == -5 or (rc == -1 and detail and (what.startswith("hl_group") or
                                                 what in ("hl_forward_record", "hl_adjoint_run"))):
            msg += ": " + detail
        raise HyperLagError(f"{what} failed: {msg} ({rc})")
    return rc


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _arg(a, dtype):
    """(pointer, keep-alive, on_device) for a numpy array or torch tensor."""
    if a is None:
        return None, None, 0
    if _is_torch(a):
        import torch
        tdt = {np.float64: torch.float64, np.int32: torch.int32, np.uint8: torch.uint8}[dtype]
        t = a.contiguous()
        if t.dtype != tdt:
            t = t.to(tdt)
        return C.c_void_p(t.data_ptr()), t, 1 if t.is_cuda else 0
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data_as(C.c_void_p), arr, 0


def mesh_check(dim, x, cells):
    """Host-side check of a simplicial mesh (hl_mesh_check): 0 if it is
    valid and conforming, else the status code (HL_E_INVALID,
    HL_E_DEGENERATE_CELL, HL_E_NONCONFORMING).  Needs no GPU."""
    xx = np.ascontiguousarray(x, dtype=np.float64)
    cc = np.ascontiguousarray(cells, dtype=np.int32)
    return int(load().hl_mesh_check(int(dim), int(xx.shape[0]), xx.ctypes.data_as(C.c_void_p),
                                    int(cc.shape[0]), cc.ctypes.data_as(C.c_void_p)))


def acoustic_dt_noalloc(x, cells, rho0, mu, lam, tau, c_cfl, out, device=0, stream=None):
    """hl_acoustic_dt_noalloc on CUDA tensors (no context, nothing
    allocated by the library): enqueues C_CFL min L_c / a_c into the
    one-element float64 tensor ``out``."""
    def p(t, dtype):
        return _arg(t, dtype)
    args = [p(a, np.float64) for a in (x, rho0, mu, lam, tau)]
    pc = p(cells, np.int32)
    po = p(out, np.float64)
    if not all(a[2] for a in args + [pc, po]):
        raise ValueError("hl_acoustic_dt_noalloc takes device arrays")
    handle = None if stream is None else C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream")
                                                    else int(stream))
    dim = int(x.shape[1])
    _check(load().hl_acoustic_dt_noalloc(int(device), handle, dim, int(x.shape[0]), args[0][0], int(cells.shape[0]),
                                         pc[0], args[1][0], args[2][0], args[3][0], args[4][0], float(c_cfl),
                                         po[0]), "hl_acoustic_dt_noalloc")
    return out


def measure_peaks(device=0, stream=None, copy_bytes=1 << 30):
    """hl_measure_peaks: (copy GB/s, FP64 FMA TFLOP/s) of two plain kernels
    on the device."""
    handle = None if stream is None else C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream")
                                                    else int(stream))
    gbs, tf = C.c_double(), C.c_double()
    _check(load().hl_measure_peaks(int(device), handle, int(copy_bytes), C.byref(gbs), C.byref(tf)),
           "hl_measure_peaks")
    return gbs.value, tf.value


class Context:
    """One mesh (or mesh batch) with its device state on one GPU."""

    def __init__(self, device=0, stream=None):
        L = load()
        self._h = C.c_void_p()
        handle = None
        if stream is not None:
            handle = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        _check(L.hl_create(C.byref(self._h), int(device), handle), "hl_create")
        self.dim = None
        self.n_nodes = self.n_cells = 0

    def close(self):
        if self._h:
            load().hl_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload_mesh(self, dim, x, cells, nwall=None, normals=None):
        px, kx, dev = _arg(x, np.float64)
        pc, kc, _ = _arg(cells, np.int32)
        pw, kw, _ = _arg(nwall, np.uint8)
        pn, kn, _ = _arg(normals, np.float64)
        nn = int(x.shape[0])
        nc = int(cells.shape[0])
        _check(load().hl_mesh_upload(self._h, int(dim), nn, px, nc, pc, pw, pn, dev),
               "hl_mesh_upload")
        self._n_contact = 0
        self.dim, self.n_nodes, self.n_cells = int(dim), nn, nc

    def set_numbering(self, numbering):
        """Internal numbering of the next uploads: NUMBERING_SPATIAL (the
        default; Hilbert order of the cells, nodes by first use) or
        NUMBERING_KEEP.  Arrays at the interface keep the caller's order."""
        _check(load().hl_set_numbering(self._h, int(numbering)), "hl_set_numbering")

    def save_state(self):
        """Snapshot of the held state (bytes)."""
        n = C.c_int64()
        _check(load().hl_state_save(self._h, None, C.byref(n)), "hl_state_save")
        buf = C.create_string_buffer(n.value)
        _check(load().hl_state_save(self._h, C.cast(buf, C.c_void_p), C.byref(n)), "hl_state_save")
        return buf.raw

    def restore_state(self, blob):
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(load().hl_state_restore(self._h, C.cast(buf, C.c_void_p), len(blob)), "hl_state_restore")

    def refine(self, levels=1):
        """Conforming red refinement of the held mesh on the GPU; the state
        is discarded (children of cell c are 8c..8c+7, 4c..4c+3 in 2D)."""
        _check(load().hl_mesh_refine(self._h, int(levels)), "hl_mesh_refine")
        d, nn, nc = C.c_int(), C.c_int64(), C.c_int64()
        _check(load().hl_mesh_info(self._h, C.byref(d), C.byref(nn), C.byref(nc)), "hl_mesh_info")
        self.dim, self.n_nodes, self.n_cells = d.value, nn.value, nc.value

    def mesh(self):
        """The held mesh in its reference configuration: x, cells, nwall,
        normals."""
        d, nn, nc = self.dim, self.n_nodes, self.n_cells
        x = np.zeros((nn, d))
        cells = np.zeros((nc, d + 1), np.int32)
        nwall = np.zeros(nn, np.uint8)
        normals = np.zeros((nn, d, d))
        _check(load().hl_mesh_get(self._h, *(a.ctypes.data_as(C.c_void_p) for a in (x, cells, nwall, normals)), 0),
               "hl_mesh_get")
        return dict(x=x, cells=cells, nwall=nwall, normals=normals)

    def upload_mesh_batch(self, dim, node_offsets, cell_offsets, x, cells, nwall=None, normals=None):
        """Concatenated meshes; ``cells`` in mesh-local node numbers."""
        no = np.ascontiguousarray(node_offsets, dtype=np.int64)
        co = np.ascontiguousarray(cell_offsets, dtype=np.int64)
        px, kx, dev = _arg(x, np.float64)
        pc, kc, _ = _arg(cells, np.int32)
        pw, kw, _ = _arg(nwall, np.uint8)
        pn, kn, _ = _arg(normals, np.float64)
        _check(load().hl_mesh_upload_batch(self._h, int(dim), len(no) - 1,
                                           no.ctypes.data_as(C.c_void_p), co.ctypes.data_as(C.c_void_p),
                                           px, pc, pw, pn, dev), "hl_mesh_upload_batch")
        self.dim, self.n_nodes, self.n_cells = int(dim), int(no[-1]), int(co[-1])
        self.n_meshes = len(no) - 1
        self.node_offsets, self.cell_offsets = no, co

    def step_batch(self, dt_per_mesh=None, info=True):
        inf = StepInfo() if info else None
        if dt_per_mesh is None:
            p, keep, dev = None, None, 0
        else:
            p, keep, dev = _arg(dt_per_mesh, np.float64)
        rc = _check(load().hl_step_batch(self._h, p, dev, C.byref(inf) if info else None),
                    "hl_step_batch")
        out = inf.as_dict() if info else {}
        out["rc"] = rc
        return out

    def next_dt(self):
        n = getattr(self, "n_meshes", 1)
        out = np.empty(n, dtype=np.float64)
        _check(load().hl_query_dt(self._h, out.ctypes.data_as(C.c_void_p), n, 0), "hl_query_dt")
        return out

    def init_state(self, rho0, mu, lam, v_cell, v_node, params=None):
        args = [_arg(a, np.float64) for a in (rho0, mu, lam, v_cell, v_node)]
        dev = args[0][2]
        prm = params if params is not None else default_params(self.dim)
        self.params = prm
        _check(load().hl_state_init(self._h, *[a[0] for a in args], C.byref(prm), dev),
               "hl_state_init")

    def set_params(self, params):
        self.params = params
        _check(load().hl_set_params(self._h, C.byref(params)), "hl_set_params")

    def set_boundary_loads(self, cell=None, face=None, kind=None, value=None):
        """Loads on boundary faces: face ``face[l]`` (opposite that local
        node) of cell ``cell[l]``; ``kind`` 1 = traction with ``value[l]`` the
        stress (11, 22, 33, 12, 13, 23), 2 = outward normal velocity
        ``value[l][0]``.  No arguments remove every load."""
        if cell is None or len(cell) == 0:
            _check(load().hl_set_boundary_loads(self._h, 0, None, None, None, None, 0),
                   "hl_set_boundary_loads")
            return
        n = len(cell)
        pc, kc, dev = _arg(cell, np.int32)
        pf, kf, df = _arg(face, np.uint8)
        pk, kk, dk = _arg(kind, np.uint8)
        pv, kv, dv = _arg(value, np.float64)
        if len(face) != n or len(kind) != n or tuple(kv.shape) != (n, 6):
            raise ValueError("cell, face, kind: [n]; value: [n][6]")
        if not dev == df == dk == dv:
            raise ValueError("boundary load arrays must all be on the host or all on the device")
        _check(load().hl_set_boundary_loads(self._h, n, pc, pf, pk, pv, dev), "hl_set_boundary_loads")

    def set_contact(self, nodes=None, point=None, normal=None):
        """Rigid-plane contact for the candidate ``nodes`` (plane through
        ``point``, ``normal`` pointing into the body).  No arguments remove
        it."""
        if nodes is None or len(nodes) == 0:
            _check(load().hl_set_contact(self._h, 0, None, None, None, 0), "hl_set_contact")
            self._n_contact = 0
            return
        pn, kn, dev = _arg(nodes, np.int32)
        pt = np.ascontiguousarray(point, dtype=np.float64)
        nr = np.ascontiguousarray(normal, dtype=np.float64)
        if pt.size < self.dim or nr.size < self.dim:
            raise ValueError("point and normal need dim components")
        _check(load().hl_set_contact(self._h, len(nodes), pn, pt.ctypes.data_as(C.c_void_p),
                                     nr.ctypes.data_as(C.c_void_p), dev), "hl_set_contact")
        self._n_contact = len(nodes)

    def contact_state(self):
        n = getattr(self, "_n_contact", 0)
        out = np.zeros(n, np.uint8)
        _check(load().hl_get_contact(self._h, out.ctypes.data_as(C.c_void_p) if n else None, n),
               "hl_get_contact")
        return out.astype(bool)

    def compute_dt(self):
        dt = C.c_double()
        _check(load().hl_compute_dt(self._h, C.byref(dt)), "hl_compute_dt")
        return dt.value

    def step(self, dt=0.0, info=True):
        inf = StepInfo() if info else None
        rc = _check(load().hl_step(self._h, float(dt), C.byref(inf) if info else None), "hl_step")
        out = inf.as_dict() if info else {}
        out["rc"] = rc
        return out

    def step_replay(self, dt, mask, info=True):
        pm, km, dev = _arg(mask, np.uint8)
        inf = StepInfo() if info else None
        rc = _check(load().hl_step_replay(self._h, float(dt), pm, dev,
                                          C.byref(inf) if info else None), "hl_step_replay")
        out = inf.as_dict() if info else {}
        out["rc"] = rc
        return out

    def _shape(self, field):
        d = self.dim
        if field in (HL_X, HL_VHAT, HL_VSTAR):
            return (self.n_nodes, d), np.float64
        if field in (HL_TAU, HL_E, HL_MASS):
            return (self.n_cells,), np.float64
        if field == HL_V:
            return (self.n_cells, d), np.float64
        if field == HL_B:
            return (self.n_cells, 6 if d == 3 else 3), np.float64
        if field == HL_ORDER:
            return (self.n_cells,), np.uint8
        if field == HL_T:
            return (self.n_cells, 6 if d == 3 else 4), np.float64
        raise ValueError(field)

    def query(self, field, out=None):
        """Return a field as a numpy array, or fill the torch tensor ``out``."""
        f = FIELDS[field] if isinstance(field, str) else int(field)
        shape, dt = self._shape(f)
        count = int(np.prod(shape))
        if out is None:
            arr = np.empty(shape, dtype=dt)
            _check(load().hl_query(self._h, f, arr.ctypes.data_as(C.c_void_p), count, 0), "hl_query")
            return arr
        p, keep, dev = _arg(out, dt)
        _check(load().hl_query(self._h, f, p, count, dev), "hl_query")
        return out

    def upload_field(self, field, values):
        f = FIELDS[field] if isinstance(field, str) else int(field)
        shape, dt = self._shape(f)
        p, keep, dev = _arg(values, dt)
        _check(load().hl_upload_field(self._h, f, p, int(np.prod(shape)), dev), "hl_upload_field")

    def state(self):
        return {k: self.query(k) for k in ("x", "vhat", "tau", "v", "e", "B")}

    def set_state(self, st):
        for k in ("x", "vhat", "tau", "v", "e", "B"):
            self.upload_field(k, st[k])

    def use_graph(self, on=True, max_mood_passes=6):
        _check(load().hl_use_graph(self._h, 1 if on else 0, int(max_mood_passes)), "hl_use_graph")

    # --------------------------------------------------------- schedules
    def set_schedule(self, stage, tile=256, block=256, blocks_per_cu=0):
        st = Schedule(int(tile), int(block), int(blocks_per_cu), 0)
        _check(load().hl_set_schedule(self._h, STAGES.index(stage), C.byref(st)), "hl_set_schedule")

    def get_schedule(self, stage):
        st = Schedule()
        _check(load().hl_get_schedule(self._h, STAGES.index(stage), C.byref(st)), "hl_get_schedule")
        return dict(tile=st.tile, block=st.block, blocks_per_cu=st.blocks_per_cu)

    def autotune(self, reps=3):
        """Pick the fastest launch schedule of every stage on the current
        mesh and state; returns {stage: (schedule, mean launch ms)}."""
        best = np.zeros(len(STAGES))
        _check(load().hl_autotune(self._h, int(reps), best.ctypes.data_as(C.c_void_p)), "hl_autotune")
        return {k: (self.get_schedule(k), float(best[i])) for i, k in enumerate(STAGES)}

    # ----------------------------------------------------------- adjoint
    def forward_record(self, nsteps, ckpt_every=20):
        _check(load().hl_forward_record(self._h, int(nsteps), int(ckpt_every)), "hl_forward_record")
        self.record_generation = getattr(self, "record_generation", 0) + 1

    def forward_replay(self):
        _check(load().hl_forward_replay(self._h), "hl_forward_replay")

    def adjoint_run(self, dL_dx):
        """Gradients (dL/dmu [n_cells], dL/dv_cell [n_cells, d], dL/dv_node
        [n_nodes, d]) for dL/dx_final; numpy in -> numpy out, CUDA tensor in
        -> CUDA tensors out."""
        d = self.dim
        if _is_torch(dL_dx) and dL_dx.is_cuda:
            import torch
            g = dL_dx.contiguous().to(torch.float64)
            mu = torch.empty(self.n_cells, dtype=torch.float64, device=g.device)
            vc = torch.empty((self.n_cells, d), dtype=torch.float64, device=g.device)
            vn = torch.empty((self.n_nodes, d), dtype=torch.float64, device=g.device)
            _check(load().hl_adjoint_run(self._h, C.c_void_p(g.data_ptr()), C.c_void_p(mu.data_ptr()),
                                         C.c_void_p(vc.data_ptr()), C.c_void_p(vn.data_ptr()), 1),
                   "hl_adjoint_run")
            return mu, vc, vn
        g = np.ascontiguousarray(dL_dx, dtype=np.float64)
        mu = np.empty(self.n_cells)
        vc = np.empty((self.n_cells, d))
        vn = np.empty((self.n_nodes, d))
        _check(load().hl_adjoint_run(self._h, g.ctypes.data_as(C.c_void_p), mu.ctypes.data_as(C.c_void_p),
                                     vc.ctypes.data_as(C.c_void_p), vn.ctypes.data_as(C.c_void_p), 0),
               "hl_adjoint_run")
        return mu, vc, vn

    def tape(self, step):
        mask = np.empty(self.n_cells, np.uint8)
        dt = np.empty(getattr(self, "n_meshes", 1))
        _check(load().hl_tape_get(self._h, int(step), mask.ctypes.data_as(C.c_void_p),
                                  dt.ctypes.data_as(C.c_void_p)), "hl_tape_get")
        return mask, dt

    # kernel timing with HIP events on the context's stream
    def profile(self, on=True):
        _check(load().hl_profile_enable(self._h, 1 if on else 0), "hl_profile_enable")

    def profile_reset(self):
        _check(load().hl_profile_reset(self._h), "hl_profile_reset")

    def profile_get(self, name):
        ms = C.c_double()
        n = C.c_int64()
        _check(load().hl_profile_get(self._h, name.encode(), C.byref(ms), C.byref(n)),
               "hl_profile_get")
        return ms.value, n.value


class Group:
    """A 2D and a 3D context stepped together (hl_group_*): each stage, MOOD
    pass and CFL reduction of the two is one kernel launch.  Holds
    references to both contexts, so they outlive it."""

    def __init__(self, ctx_2d, ctx_3d):
        self._h = C.c_void_p()
        self.contexts = (ctx_2d, ctx_3d)
        _check(load().hl_group_create(C.byref(self._h), ctx_2d._h, ctx_3d._h), "hl_group_create")

    def close(self):
        if self._h:
            load().hl_group_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def use_graph(self, on=True, max_mood_passes=6):
        _check(load().hl_group_use_graph(self._h, 1 if on else 0, int(max_mood_passes)), "hl_group_use_graph")

    def step(self, info=True):
        """One step of both contexts on their device-held dt; returns the
        two step reports (2D, 3D)."""
        i2 = StepInfo() if info else None
        i3 = StepInfo() if info else None
        rc = _check(load().hl_group_step(self._h, C.byref(i2) if info else None, C.byref(i3) if info else None),
                    "hl_group_step")
        out = (i2.as_dict() if info else {}, i3.as_dict() if info else {})
        for o in out:
            o["rc"] = rc
        return out


def from_workloads(ws, device=0, stream=None, params=None):
    """One batched context from several workloads of the same dimension."""
    dims = {w.dim for w in ws}
    if len(dims) != 1:
        raise ValueError("a batch holds meshes of one dimension")
    dim = dims.pop()
    no = np.concatenate([[0], np.cumsum([w.n_nodes for w in ws])])
    co = np.concatenate([[0], np.cumsum([w.n_cells for w in ws])])
    cat = lambda f: np.concatenate([getattr(w, f) for w in ws])
    ctx = Context(device, stream)
    ctx.upload_mesh_batch(dim, no, co, cat("x"), cat("cells"), cat("nwall"), cat("normals"))
    init_from_workloads(ctx, ws, params)
    return ctx


def init_from_workloads(ctx, ws, params=None):
    """(Re)initialise the state of a batched context built from ``ws``."""
    cat = lambda f: np.concatenate([getattr(w, f) for w in ws])
    ctx.init_state(cat("rho0"), cat("mu"), cat("lam"), cat("v_cell"), cat("v_node"),
                   params if params is not None else default_params(ws[0].dim, c_cfl=ws[0].c_cfl))


def from_workload(w, device=0, stream=None, params=None):
    """Context initialised from a ``workloads.Workload``."""
    ctx = Context(device, stream)
    ctx.upload_mesh(w.dim, w.x, w.cells, w.nwall, w.normals)
    ctx.init_state(w.rho0, w.mu, w.lam, w.v_cell, w.v_node,
                   params if params is not None else default_params(w.dim, c_cfl=w.c_cfl))
    return ctx
