"""ctypes binding of the FP64 CPU oracle (``oracle/hl_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``.
The HIP library never imports or links anything from here.

All arrays follow the layout of the C-ABI of the library: node vectors
``[n_nodes, dim]``, cell vectors ``[n_cells, dim]``, B as ``[n_cells, nB]``
with components (11, 22, 33, 12, 13, 23) in 3D and (11, 22, 12) in 2D.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hl_oracle.c")
LIB = os.path.join(HERE, "libhl_oracle.so")
# the same source threaded over output cells and nodes (OpenMP), for the
# timed CPU baseline only; bitwise the serial results
LIB_OMP = os.path.join(HERE, "libhl_oracle_omp.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared",
          "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas", "-Wno-maybe-uninitialized"]
CFLAGS_OMP = ["-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared",
              "-Wall", "-Wno-unused-function", "-Wno-maybe-uninitialized"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction): the serial
    library and its OpenMP build."""
    for lib_path, flags in ((LIB, CFLAGS), (LIB_OMP, CFLAGS_OMP)):
        if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(SRC):
            tmp = lib_path + ".tmp"
            subprocess.check_call(["gcc", *flags, SRC, "-o", tmp, "-lm"])
            os.replace(tmp, lib_path)
    return LIB


_variant = "serial"


def use_threads(on: bool) -> None:
    """Select the OpenMP build (True) or the serial one (False) for the
    libraries loaded from now on; call before the first oracle call."""
    global _variant, _lib
    want = "omp" if on else "serial"
    if want != _variant:
        _variant = want
        _lib = None


class Params(C.Structure):
    _fields_ = [("c_cfl", C.c_double), ("c_v", C.c_double), ("c_i", C.c_double),
                ("delta0", C.c_double), ("delta1", C.c_double), ("eps_tol", C.c_double),
                ("detect", C.c_int), ("cascade", C.c_int), ("shear_a", C.c_double),
                ("eos", C.c_int), ("pad_", C.c_int), ("sg_gamma", C.c_double), ("sg_pinf", C.c_double)]


class Info(C.Structure):
    _fields_ = [("dt_next", C.c_double), ("dt_acoustic", C.c_double),
                ("dt_volume", C.c_double), ("mass", C.c_double), ("mom", C.c_double * 3),
                ("energy", C.c_double), ("kinetic", C.c_double), ("elastic", C.c_double),
                ("n_p0", C.c_int64), ("n_flag_first", C.c_int64), ("mood_iters", C.c_int32),
                ("status", C.c_int32), ("n_lim", C.c_int64), ("n_recomp", C.c_int64),
                ("gcl_defect", C.c_double), ("detB_defect", C.c_double), ("n_detB", C.c_int64)]

    def as_dict(self):
        return dict(dt_next=self.dt_next, dt_acoustic=self.dt_acoustic,
                    dt_volume=self.dt_volume, mass=self.mass, mom=list(self.mom),
                    energy=self.energy, kinetic=self.kinetic, elastic=self.elastic,
                    n_p0=self.n_p0, n_flag_first=self.n_flag_first,
                    mood_iters=self.mood_iters, status=self.status, n_lim=self.n_lim,
                    n_recomp=self.n_recomp, gcl_defect=self.gcl_defect,
                    detB_defect=self.detB_defect, n_detB=self.n_detB)


def default_params(c_cfl=0.25, detect=True, cascade=2, shear_a=-1.0, eos=0, sg_gamma=2.2, sg_pinf=1e6):
    """Paper values: C_v = 0.2, C_i = 0.1, delta0 = 1e-4, delta1 = 1e-3
    (Sections 3.5 and 3.6).  cascade 2: P1 -> P0; 3: P1 -> P1 with the
    Barth-Jespersen limiter -> P0 (Section 3.5).  shear_a: parameter of the
    shear energy family (eq. familiy_energies); -1 is neo-Hookean.  eos 1:
    the stiffened gas (eq. EOS_stiffened_gas) with gamma and p_inf (the
    droplet test's 2.2 and 1e6 by default) in place of the volumetric
    energy of eq. EOS_neoHook."""
    return Params(c_cfl, 0.2, 0.1, 1e-4, 1e-3, 1e-12, 1 if detect else 0, int(cascade), float(shear_a),
                  int(eos), 0, float(sg_gamma), float(sg_pinf))


_lib = None
_P = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_U8 = C.POINTER(C.c_uint8)


def lib():
    global _lib
    if _lib is None:
        path = LIB_OMP if _variant == "omp" else LIB
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        L.orc_mesh_new.restype = C.c_void_p
        L.orc_mesh_new.argtypes = [C.c_int, C.c_int64, C.c_int64, _I32, _U8, _P]
        L.orc_mesh_free.argtypes = [C.c_void_p]
        L.orc_set_loads.restype = C.c_int
        L.orc_set_loads.argtypes = [C.c_void_p, C.c_int64, _I32, _U8, _U8, _P]
        L.orc_set_node_walls.restype = C.c_int
        L.orc_set_node_walls.argtypes = [C.c_void_p, C.c_int64, C.c_int, _P]
        L.orc_init_state.restype = C.c_int
        L.orc_init_state.argtypes = [C.c_void_p] + [_P] * 6 + [_P] * 7
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = ([C.c_void_p] + [_P] * 4 + [_P] * 6 + [C.c_double, C.POINTER(Params),
                               _U8, C.c_int] + [_P] * 7 + [C.POINTER(Info)])
        L.orc_initial_dt.restype = C.c_double
        L.orc_initial_dt.argtypes = [C.c_void_p] + [_P] * 9 + [C.POINTER(Params)]
        L.orc_cell_geometry.argtypes = [C.c_int, _P, _P, _P, _P, _P, _P]
        L.orc_corner_shape.argtypes = [C.c_int, _P, C.c_int, _P]
        L.orc_point_stress.argtypes = [C.c_double] * 4 + [_P, _P, _P, _P, _P, C.c_double]
        L.orc_point_stress_direction.argtypes = [C.c_double] * 4 + [_P, C.c_double, _P, _P, C.c_double]
        L.orc_point_cn.restype = C.c_int
        L.orc_point_cn.argtypes = [C.c_int, _P, _P, _P, C.c_double, _P]
        L.orc_lsq.argtypes = [C.c_void_p] + [_P] * 5
        L.orc_bj.argtypes = [C.c_void_p] + [_P] * 5
        L.orc_predict.argtypes = ([C.c_void_p] + [_P] * 7 + [C.c_double, C.c_double, _U8] + [_P] * 5)
        L.orc_diagnostics.argtypes = [C.c_void_p] + [_P] * 8 + [C.POINTER(Info), C.POINTER(Params)]
        L.orc_predict_eos.argtypes = ([C.c_void_p] + [_P] * 8 + [C.c_double, C.POINTER(Params), _U8] + [_P] * 4)
        L.orc_point_stress_sg.argtypes = [C.c_double] * 6 + [_P, C.c_double, _P, _P, _P, _P]
        L.orc_point_stress_direction_sg.argtypes = ([C.c_double] * 6 + [_P, C.c_double, C.c_double, _P,
                                                    C.c_double, _P])
        L.orc_detect.argtypes = [C.c_void_p] + [_P] * 8 + [_U8, C.POINTER(Params), _U8]
        L.orc_time_step.argtypes = ([C.c_void_p] + [_P] * 10 + [C.c_double, C.POINTER(Params),
                                    C.POINTER(Info)])
        L.orc_info_size.restype = C.c_int
        L.orc_params_size.restype = C.c_int
        assert L.orc_info_size() == C.sizeof(Info)
        assert L.orc_params_size() == C.sizeof(Params)
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_P)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_P)


# -------------------------------------------------------------- point-wise

def cell_geometry(X):
    """X: [(d+1), d] vertex coordinates -> dict(V, xc, C, A, Lc)."""
    X = _f64(X)
    d = X.shape[1]
    V = np.zeros(1)
    Lc = np.zeros(1)
    xc = np.zeros(3)
    Cc = np.zeros((d + 1, 3))
    A = np.zeros((d + 1, 3))
    lib().orc_cell_geometry(d, _ptr(X), _ptr(V), _ptr(xc), _ptr(Cc), _ptr(A), _ptr(Lc))
    return dict(V=V[0], xc=xc[:d], C=Cc[:, :d], A=A[:, :d], Lc=Lc[0])


def corner_shape(X, p):
    X = _f64(X)
    N = np.zeros((3, 3))
    lib().orc_corner_shape(X.shape[1], _ptr(X), int(p), _ptr(N))
    return N


def point_stress(rho0, mu, K, tau, B, shear_a=-1.0):
    """Full 3x3 B -> (T 3x3, p, a, Psi); shear_a selects the shear energy
    of the family (eq. familiy_energies), -1 neo-Hookean."""
    B = _f64(B)
    T = np.zeros((3, 3))
    p = np.zeros(1)
    a = np.zeros(1)
    psi = np.zeros(1)
    lib().orc_point_stress(rho0, mu, K, tau, _ptr(B), _ptr(T), _ptr(p), _ptr(a), _ptr(psi), float(shear_a))
    return T, p[0], a[0], psi[0]


def point_stress_sg(rho0, mu, tau, B, eps, shear_a=-1.0, gamma=2.2, p_inf=1e6):
    """Stiffened gas with the shear family (eq. EOS_stiffened_gas; R31):
    (T, p, a, Psi_s) at (tau, B, eps), eps the specific internal energy."""
    T = np.zeros(9)
    p, a, psi = C.c_double(), C.c_double(), C.c_double()
    lib().orc_point_stress_sg(rho0, mu, shear_a, gamma, p_inf, tau, _ptr(_f64(np.reshape(B, 9))), eps,
                              _ptr(T), C.byref(p), C.byref(a), C.byref(psi))
    return T.reshape(3, 3), p.value, a.value, psi.value


def point_stress_direction_sg(rho0, mu, tau, B, eps, dtau, dB, deps, shear_a=-1.0, gamma=2.2, p_inf=1e6):
    dT = np.zeros(9)
    lib().orc_point_stress_direction_sg(rho0, mu, shear_a, gamma, p_inf, tau, _ptr(_f64(np.reshape(B, 9))), eps,
                                        dtau, _ptr(_f64(np.reshape(dB, 9))), deps, _ptr(dT))
    return dT.reshape(3, 3)


def point_stress_direction(rho0, mu, K, tau, B, dtau, dB, shear_a=-1.0):
    B = _f64(B)
    dB = _f64(dB)
    dT = np.zeros((3, 3))
    lib().orc_point_stress_direction(rho0, mu, K, tau, _ptr(B), dtau, _ptr(dB), _ptr(dT), float(shear_a))
    return dT


def point_cn(d, Bn, Ln, L1, dt):
    Bn, Ln, L1 = _f64(Bn), _f64(Ln), _f64(L1)
    out = np.zeros((3, 3))
    st = lib().orc_point_cn(d, _ptr(Bn), _ptr(Ln), _ptr(L1), dt, _ptr(out))
    assert st == 0
    return out


# -------------------------------------------------------------- mesh level

@dataclass
class State:
    x: np.ndarray
    vhat: np.ndarray
    tau: np.ndarray
    v: np.ndarray
    e: np.ndarray
    B: np.ndarray

    def copy(self):
        return State(*(np.array(a, copy=True) for a in
                       (self.x, self.vhat, self.tau, self.v, self.e, self.B)))


class Mesh:
    """Oracle mesh: connectivity, node->corner lists and wall bases."""

    def __init__(self, dim, x, cells, nwall=None, normals=None):
        self.dim = int(dim)
        self.cells = np.ascontiguousarray(cells, dtype=np.int32)
        self.nn = int(np.asarray(x).shape[0])
        self.nc = int(self.cells.shape[0])
        self.nB = 6 if dim == 3 else 3
        if nwall is None:
            nwall = np.zeros(self.nn, np.uint8)
        if normals is None:
            normals = np.zeros((self.nn, dim, dim))
        self._nwall = np.ascontiguousarray(nwall, dtype=np.uint8)
        self._normals = _f64(normals)
        h = lib().orc_mesh_new(self.dim, self.nn, self.nc, self.cells.ctypes.data_as(_I32),
                               self._nwall.ctypes.data_as(_U8), _ptr(self._normals))
        if not h:
            raise ValueError("invalid mesh")
        self.h = h

    def set_loads(self, cell, face, kind, value):
        """Boundary loads (Appendix B): face (cell, k) is the face opposite
        the cell's k-th node; kind 1 traction tensor value[6] in (11, 22,
        33, 12, 13, 23) order, kind 2 normal velocity value[0]."""
        self._ld = (np.ascontiguousarray(cell, np.int32), np.ascontiguousarray(face, np.uint8),
                    np.ascontiguousarray(kind, np.uint8), _f64(np.reshape(value, (-1, 6))))
        rc = lib().orc_set_loads(self.h, len(self._ld[0]), self._ld[0].ctypes.data_as(_I32),
                                 self._ld[1].ctypes.data_as(_U8), self._ld[2].ctypes.data_as(_U8),
                                 _ptr(self._ld[3]))
        if rc != 0:
            raise ValueError("invalid boundary load")

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.orc_mesh_free(h)
            self.h = None


class Problem:
    """Mesh + material + state, advanced by the oracle."""

    def __init__(self, w, params=None):
        self.w = w
        self.dim = w.dim
        self.mesh = Mesh(w.dim, w.x, w.cells, w.nwall, w.normals)
        nc, nn, d = w.n_cells, w.n_nodes, w.dim
        self.rho0 = _f64(w.rho0)
        self.mu = _f64(w.mu)
        lam = _f64(w.lam)
        self.m = np.zeros(nc)
        self.K = np.zeros(nc)
        st = State(_f64(w.x).copy(), np.zeros((nn, d)), np.zeros(nc), np.zeros((nc, d)),
                   np.zeros(nc), np.zeros((nc, self.mesh.nB)))
        vc, vn = _f64(w.v_cell), _f64(w.v_node)
        rc = lib().orc_init_state(self.mesh.h, _ptr(st.x), _ptr(self.rho0), _ptr(self.mu),
                                  _ptr(lam), _ptr(vc), _ptr(vn), _ptr(self.m), _ptr(self.K),
                                  _ptr(st.tau), _ptr(st.v), _ptr(st.e), _ptr(st.B),
                                  _ptr(st.vhat))
        if rc != 0:
            raise ValueError("degenerate cell in the initial mesh")
        self.params = params if params is not None else default_params(w.c_cfl)
        if self.params.eos == 1:
            # stiffened gas at rest pressure p = 0 (reading R31):
            # e = |v|^2 / 2 + gamma p_inf tau / (gamma - 1), Psi_s(B = I) = 0
            g, pinf = self.params.sg_gamma, self.params.sg_pinf
            st.e = st.e + g * pinf * st.tau / (g - 1.0)
        self.state = st
        self.dt_prev = 0.0
        self.t = 0.0

    def initial_dt(self):
        s = self.state
        ins = [_f64(a) for a in (s.x, s.tau, s.v, s.e, s.B)]
        return lib().orc_initial_dt(self.mesh.h, _ptr(self.rho0), _ptr(self.mu), _ptr(self.K),
                                    *[_ptr(a) for a in ins], _ptr(self.m), C.byref(self.params))

    def step(self, dt, mask=None, replay=False, state=None):
        """Advance ``state`` (default: the held state) by ``dt``.  Returns
        (new_state, vstar, mask, info); the held state is replaced only when
        ``state`` is None."""
        s = self.state if state is None else state
        nc, nn, d = self.mesh.nc, self.mesh.nn, self.dim
        mk = np.zeros(nc, np.uint8) if mask is None else np.array(mask, dtype=np.uint8, copy=True)
        out = State(np.zeros((nn, d)), np.zeros((nn, d)), np.zeros(nc), np.zeros((nc, d)),
                    np.zeros(nc), np.zeros((nc, self.mesh.nB)))
        vstar = np.zeros((nn, d))
        info = Info()
        ins = [_f64(a) for a in (s.x, s.vhat, s.tau, s.v, s.e, s.B)]
        lib().orc_step(self.mesh.h, _ptr(self.rho0), _ptr(self.mu), _ptr(self.K), _ptr(self.m),
                       *[_ptr(a) for a in ins], float(dt), C.byref(self.params),
                       mk.ctypes.data_as(_U8), 1 if replay else 0,
                       _ptr(out.x), _ptr(out.vhat), _ptr(out.tau), _ptr(out.v), _ptr(out.e),
                       _ptr(out.B), _ptr(vstar), C.byref(info))
        if state is None:
            self.state = out
            self.t += dt
            self.dt_prev = dt
        return out, vstar, mk, info

    def run(self, steps, dt=None, callback=None):
        """Advance ``steps`` steps with CFL control (or a fixed ``dt``)."""
        dt_next = self.initial_dt() if dt is None else dt
        infos = []
        for _ in range(steps):
            cur = dt_next
            _, _, mk, info = self.step(cur)
            infos.append(info.as_dict())
            if callback:
                callback(self, mk, info)
            dt_next = info.dt_next if dt is None else dt
        return infos

    def lsq(self, state=None):
        s = self.state if state is None else state
        g = np.zeros((self.mesh.nc, 1 + self.dim + self.mesh.nB, 3))
        ins = [_f64(a) for a in (s.x, s.tau, s.v, s.B)]
        lib().orc_lsq(self.mesh.h, *[_ptr(a) for a in ins], _ptr(g))
        return g[:, :, :self.dim]

    def bj(self, state=None):
        """Barth-Jespersen limited gradients [nc, nW, d] (Section 3.5)."""
        s = self.state if state is None else state
        g = np.zeros((self.mesh.nc, 1 + self.dim + self.mesh.nB, 3))
        ins = [_f64(a) for a in (s.x, s.tau, s.v, s.B)]
        lib().orc_bj(self.mesh.h, *[_ptr(a) for a in ins], _ptr(g))
        return g[:, :, :self.dim]

    def predict(self, dt, mask=None, state=None):
        s = self.state if state is None else state
        nq = self.mesh.nc * (self.dim + 1)
        mk = np.zeros(self.mesh.nc, np.uint8) if mask is None else np.asarray(mask, np.uint8)
        tau_s, v_s = np.zeros(nq), np.zeros((nq, 3))
        B_s, T_s, z_s = np.zeros((nq, 3, 3)), np.zeros((nq, 3, 3)), np.zeros(nq)
        ins = [_f64(a) for a in (s.x, s.tau, s.v, s.B)]
        lib().orc_predict(self.mesh.h, _ptr(self.rho0), _ptr(self.mu), _ptr(self.K),
                          *[_ptr(a) for a in ins], float(dt), float(self.params.shear_a), mk.ctypes.data_as(_U8),
                          _ptr(tau_s), _ptr(v_s), _ptr(B_s), _ptr(T_s), _ptr(z_s))
        return dict(tau=tau_s, v=v_s, B=B_s, T=T_s, z=z_s)

    def predict_eos(self, dt, mask=None, state=None):
        """Corner states with this problem's equation of state: (tau*,
        eps*, T* [.., 3, 3], z*), each [n_cells, nv, ...]."""
        s = self.state if state is None else state
        nc, nv = self.mesh.nc, self.dim + 1
        mk = np.zeros(nc, np.uint8) if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        ts, es, zs = np.zeros(nc * nv), np.zeros(nc * nv), np.zeros(nc * nv)
        Ts = np.zeros(nc * nv * 9)
        ins = [_f64(a) for a in (s.x, s.tau, s.v, s.e, s.B)]
        lib().orc_predict_eos(self.mesh.h, _ptr(self.rho0), _ptr(self.mu), _ptr(self.K), *[_ptr(a) for a in ins],
                              float(dt), C.byref(self.params), mk.ctypes.data_as(_U8), _ptr(ts), _ptr(es),
                              _ptr(Ts), _ptr(zs))
        return ts.reshape(nc, nv), es.reshape(nc, nv), Ts.reshape(nc, nv, 3, 3), zs.reshape(nc, nv)

    def detect(self, cand, state=None, mask=None):
        """Detection (eqs. PAD and RDMP) of the candidate state ``cand``
        against the relaxed-DMP bounds of ``state`` (default: the held
        state): per cell 0 accepted, 1 not physically admissible, 2 outside
        the relaxed DMP bounds (cells with mask >= 2 are accepted)."""
        s = self.state if state is None else state
        nc = self.mesh.nc
        code = np.zeros(nc, np.uint8)
        mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        ins = [_f64(a) for a in (s.tau, cand.tau, cand.v, cand.e, cand.B)]
        lib().orc_detect(self.mesh.h, _ptr(self.rho0), _ptr(self.mu), _ptr(self.K), *[_ptr(a) for a in ins],
                         mk.ctypes.data_as(_U8) if mk is not None else None, C.byref(self.params),
                         code.ctypes.data_as(_U8))
        return code

    def time_step(self, cand, dt_prev, V0=None):
        """Time-step control (eqs. CFL, CFL2) of the end-of-step state
        ``cand`` after a step of ``dt_prev`` from cell volumes ``V0`` (None:
        the first step, acoustic bound only).  Returns the Info."""
        info = Info()
        ins = [_f64(a) for a in (cand.x, cand.tau, cand.v, cand.e, cand.B)]
        v0 = None if V0 is None else _f64(V0)
        lib().orc_time_step(self.mesh.h, _ptr(self.rho0), _ptr(self.mu), _ptr(self.K), *[_ptr(a) for a in ins],
                            _ptr(self.m), _ptr(v0) if v0 is not None else None, float(dt_prev),
                            C.byref(self.params), C.byref(info))
        return info

    def diagnostics(self, state=None):
        s = self.state if state is None else state
        info = Info()
        ins = [_f64(a) for a in (s.tau, s.v, s.e, s.B)]
        lib().orc_diagnostics(self.mesh.h, _ptr(self.rho0), _ptr(self.mu), _ptr(self.K),
                              _ptr(self.m), *[_ptr(a) for a in ins], C.byref(info), C.byref(self.params))
        return info.as_dict()


class Contact:
    """Rigid-plane contact with boundary conditions that change type during
    the run (Section 3.8, "Boundary condition treatments"; reading R30).

    The plane passes through ``point`` with unit ``normal`` pointing from
    the obstacle into the body.  Each candidate node is free (its own walls
    only) until it would cross the plane, then a slip wall along the plane
    (added to its own walls) until its free velocity points away from the
    plane.  One step (``step``):

    1. a trial step from t^n with the current dt and node conditions;
    2. detachment: a node in contact whose free velocity -- the nodal
       solution with its own walls only, from the same corner values --
       has a positive normal component leaves the plane at t^n; the trial
       is repeated with the same dt;
    3. impact: a free node that ends below the plane (g1 < 0, gap
       g = (x - x_T) . n) reaches it at the fraction s = g0 / (g0 - g1) of
       the step (s = 0 if g0 <= 0).  If min s <= 1e-9 those nodes go into
       contact at once and the trial is repeated; otherwise dt is cut to
       s_min dt, the nodes with s <= s_min (1 + 1e-9) are held pending (and
       left out of the check), and the trial is repeated;
    4. otherwise the trial is accepted and pending nodes go into contact
       from the next step on.  After at most 8 trials the last is accepted
       and every node still below the plane goes into contact.

    After a cut step the next dt is min(acoustic, volume, (1 + C_i) dt of
    the uncut trial), so the growth bound does not restart from the cut.
    """

    S_EPS = 1e-9
    TIE = 1e-9
    MAX_TRIALS = 8

    def __init__(self, problem, nodes, point, normal):
        self.P = problem
        d = problem.dim
        self.nodes = np.asarray(nodes, dtype=np.int64)
        self.xT = _f64(point)[:d].copy()
        n = _f64(normal)[:d]
        self.n = n / np.sqrt(np.sum(n * n))
        self.contact = np.zeros(len(self.nodes), bool)
        w = problem.w
        self.own = [np.array(w.normals[p][:int(w.nwall[p])], dtype=np.float64).reshape(-1, d)
                    for p in self.nodes]

    def _set(self, i, on):
        rows = self.own[i]
        if on and rows.shape[0] < self.P.dim:
            rows = np.vstack([rows, self.n[None, :]])
        rows = np.ascontiguousarray(rows, dtype=np.float64)
        rc = lib().orc_set_node_walls(self.P.mesh.h, int(self.nodes[i]), rows.shape[0],
                                      _ptr(rows) if rows.size else None)
        assert rc == 0

    def _apply(self):
        for i in range(len(self.nodes)):
            self._set(i, bool(self.contact[i]))

    def step(self, dt):
        """Advance the held state; returns (state, vstar, mask, info,
        report) with report = dict(dt, dt_next, trials, clipped)."""
        P = self.P
        s0 = P.state
        dt_req = dt
        pending = np.zeros(len(self.nodes), bool)
        clipped = False
        self._apply()
        for trial in range(1, self.MAX_TRIALS + 1):
            s1, vs, mk, info = P.step(dt, state=s0)
            if trial == self.MAX_TRIALS:
                break
            idx = np.nonzero(self.contact)[0]
            if len(idx):
                for i in idx:
                    self._set(i, False)
                _, vfree, _, _ = P.step(dt, mask=mk, replay=True, state=s0)
                for i in idx:
                    self._set(i, True)
                away = vfree[self.nodes[idx]] @ self.n > 0.0
                if away.any():
                    for i in idx[away]:
                        self.contact[i] = False
                        self._set(i, False)
                    continue
            g0 = (s0.x[self.nodes] - self.xT) @ self.n
            g1 = (s1.x[self.nodes] - self.xT) @ self.n
            hit = ~self.contact & ~pending & (g1 < 0.0)
            if not hit.any():
                break
            frac = np.where(g0 > 0.0, g0 / np.where(hit, g0 - g1, 1.0), 0.0)
            smin = frac[hit].min()
            if smin <= self.S_EPS:
                for i in np.nonzero(hit & (frac <= self.S_EPS))[0]:
                    self.contact[i] = True
                    self._set(i, True)
                continue
            pending |= hit & (frac <= smin * (1.0 + self.TIE))
            dt = smin * dt
            clipped = True
        if trial == self.MAX_TRIALS:
            g1 = (s1.x[self.nodes] - self.xT) @ self.n
            pending |= ~self.contact & (g1 < 0.0)
        P.state = s1
        P.t += dt
        P.dt_prev = dt
        self.contact |= pending
        self._apply()
        dt_next = info.dt_next
        if clipped:
            dt_next = min(info.dt_acoustic, info.dt_volume, (1.0 + P.params.c_i) * dt_req)
        return s1, vs, mk, info, dict(dt=dt, dt_next=dt_next, trials=trial, clipped=clipped)


def refine(dim, x, cells, nwall, normals, levels=1):
    """Conforming red refinement, ``levels`` times (Section 3.9: the local
    1 -> 8 split of every tetrahedron; 1 -> 4 for triangles), in plain
    Python over the cells.  Conventions (they fix the numbering):

    - edges are numbered in increasing (min node, max node) order; the
      midpoint of edge e is node nn + e, at 0.5 (x_p + x_q);
    - a midpoint keeps the wall normals of its first end node (the smaller
      number) that the other end node also has (unit normals with dot
      product >= 1 - 1e-12), at most dim of them;
    - the children of cell c are 8c .. 8c+7: the corner tetrahedra at v0,
      v1, v2, v3, each made of its vertex and the midpoints of its three
      edges in the parent's vertex order, then the four tetrahedra around
      the shortest diagonal of the inner octahedron -- diagonal
      (m01, m23), (m02, m13) or (m03, m12), the first if lengths tie --
      each made of the diagonal and two consecutive midpoints of the cycle
      of the other four: the cycle starts at the first of them in edge
      order (01, 02, 03, 12, 13, 23) and each next one is the first
      remaining whose edge shares a vertex of the parent with the last;
    - in 2D the children are 4c .. 4c+3: (v0, m01, m02), (m01, v1, m12),
      (m02, m12, v2), (m01, m12, m02);
    - a child of negative measure has its last two nodes swapped.
    """
    x = np.array(x, dtype=np.float64)
    cells = np.array(cells, dtype=np.int64)
    nwall = np.array(nwall, dtype=np.uint8)
    normals = np.array(normals, dtype=np.float64).reshape(len(x), dim, dim)
    for _ in range(levels):
        x, cells, nwall, normals = _refine_once(dim, x, cells, nwall, normals)
    return x, cells.astype(np.int32), nwall, normals


def _measure(dim, P):
    e = [[P[k + 1][j] - P[0][j] for j in range(dim)] for k in range(dim)]
    if dim == 2:
        return e[0][0] * e[1][1] - e[0][1] * e[1][0]
    return (e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0])
            + e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]))


def _refine_once(dim, x, cells, nwall, normals):
    nn = len(x)
    nv = dim + 1
    keys = set()
    for c in cells:
        for a in range(nv):
            for b in range(a + 1, nv):
                p, q = int(c[a]), int(c[b])
                keys.add((min(p, q), max(p, q)))
    order = sorted(keys)
    eid = {k: i for i, k in enumerate(order)}
    ne = len(order)
    xo = np.zeros((nn + ne, dim))
    xo[:nn] = x
    nw = np.zeros(nn + ne, np.uint8)
    nr = np.zeros((nn + ne, dim, dim))
    nw[:nn] = nwall
    nr[:nn] = normals
    for (p, q), e in eid.items():
        for j in range(dim):
            xo[nn + e, j] = 0.5 * (x[p, j] + x[q, j])
        cnt = 0
        for r in range(int(nwall[p])):
            n_p = normals[p, r]
            if any(float(np.dot(n_p, normals[q, t])) >= 1.0 - 1e-12 for t in range(int(nwall[q]))) and cnt < dim:
                nr[nn + e, cnt] = n_p
                cnt += 1
        nw[nn + e] = cnt

    def mid(c, a, b):
        p, q = int(c[a]), int(c[b])
        return nn + eid[(min(p, q), max(p, q))]

    def put(out, nodes):
        nodes = list(nodes)
        if _measure(dim, [xo[k] for k in nodes]) < 0.0:
            nodes[-2], nodes[-1] = nodes[-1], nodes[-2]
        out.append(nodes)

    out = []
    for c in cells:
        v = [int(k) for k in c]
        if dim == 2:
            m01, m02, m12 = mid(c, 0, 1), mid(c, 0, 2), mid(c, 1, 2)
            for t in ((v[0], m01, m02), (m01, v[1], m12), (m02, m12, v[2]), (m01, m12, m02)):
                put(out, t)
            continue
        m = {(a, b): mid(c, a, b) for a in range(4) for b in range(a + 1, 4)}
        for k in range(4):
            put(out, [v[k] if j == k else m[(min(j, k), max(j, k))] for j in range(4)])
        diags = [((0, 1), (2, 3)), ((0, 2), (1, 3)), ((0, 3), (1, 2))]

        def sq(a, b):
            d = [xo[m[a]][j] - xo[m[b]][j] for j in range(3)]
            return d[0] * d[0] + d[1] * d[1] + d[2] * d[2]

        lens = [sq(a, b) for a, b in diags]
        i = min(range(3), key=lambda t: (lens[t], t))
        da, db = diags[i]
        rest = [e for e in m if e not in (da, db)]
        # cycle of the other four: consecutive midpoints share a parent vertex
        cyc = [rest[0]]
        while len(cyc) < 4:
            nxt = [e for e in rest if e not in cyc and set(e) & set(cyc[-1])]
            cyc.append(nxt[0])
        for j in range(4):
            put(out, [m[da], m[db], m[cyc[j]], m[cyc[(j + 1) % 4]]])
    return xo, np.array(out, dtype=np.int64), nw, nr
