"""Pins of the oracle's boundary loads (Appendix B, Section 3.6 "Boundary
condition treatments"; readings R28, R29).  Expected values come from face
geometry computed here in numpy and from mechanics: a uniformly stressed
body loaded by the same stress on its boundary is in equilibrium; the
momentum and total energy of the body change by the impulse and the work of
the applied tractions; a prescribed normal velocity is met exactly at every
loaded node, and a zero one is the slip wall of the same plane; a wall
takes precedence over a velocity load."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import workloads as W


def boundary_faces(cells):
    """(cell, k) of every face that belongs to one cell; face k is opposite
    the cell's k-th node."""
    nv = cells.shape[1]
    seen = {}
    for c in range(cells.shape[0]):
        for k in range(nv):
            key = tuple(sorted(np.delete(cells[c], k)))
            seen.setdefault(key, []).append((c, k))
    return [v[0] for v in seen.values() if len(v) == 1]


def face_vector(x, cells, c, k):
    """(|f|/d) n_f, outward from cell c, of the face opposite node k."""
    d = x.shape[1]
    X = x[cells[c]]
    F = np.delete(X, k, axis=0)
    if d == 3:
        A = 0.5 * np.cross(F[1] - F[0], F[2] - F[0])
    else:
        t = F[1] - F[0]
        A = np.array([t[1], -t[0]])
    if np.dot(A, F.mean(axis=0) - X[k]) < 0:
        A = -A
    return A / d


def _sym6(T):
    return np.array([T[0, 0], T[1, 1], T[2, 2], T[0, 1], T[0, 2], T[1, 2]])


def _prestressed(w, J):
    P = O.Problem(w, O.default_params(w.c_cfl, detect=False))
    s = P.state
    s.tau[:] = J / P.rho0
    s.v[:] = 0.0
    s.vhat[:] = 0.0
    s.e[:] = 0.0
    s.B[:] = 0.0
    s.B[:, :w.dim] = J ** (2.0 / 3.0)
    return P


def _free_square():
    w = W.plane_wave_2d(n=6, amp=0.0, seed=4)
    w.nwall = np.zeros_like(w.nwall)        # no slip walls: a free body
    w.normals = np.zeros_like(w.normals)
    return w


CASES = {"tet": lambda: W.rotating_cube_3d(n=3, seed=4), "tri": _free_square}


@pytest.mark.parametrize("case", list(CASES))
def test_matching_traction_keeps_a_stressed_body_at_rest(case):
    w = CASES[case]()
    J = 0.97
    P = _prestressed(w, J)
    B3 = np.eye(3)
    B3[:w.dim, :w.dim] *= J ** (2.0 / 3.0)
    T, p, a, _ = O.point_stress(P.rho0[0], P.mu[0], P.K[0], J / P.rho0[0], B3)
    faces = boundary_faces(w.cells)
    dt = P.initial_dt()
    _, vs_free, _, _ = P.step(dt, state=P.state)
    P.mesh.set_loads([f[0] for f in faces], [f[1] for f in faces], np.ones(len(faces)),
                     np.tile(_sym6(T), (len(faces), 1)))
    s1, vs, _, _ = P.step(dt, state=P.state)
    scale = abs(p) / (P.rho0[0] * a)            # velocity of a pressure jump p
    assert np.abs(vs_free).max() > 1e-3 * scale
    assert np.abs(vs).max() <= 1e-12 * scale
    assert np.array_equal(s1.x, P.state.x + dt * vs)


def test_traction_momentum_and_energy_balance():
    """Shear traction on the top face of a free cube at rest: the change of
    momentum is dt sum_p F_p and that of total energy dt sum_p F_p . v*_p,
    with F_p = sum over loaded faces through p of T^BC (|f|/d) n_f."""
    w = W.rotating_cube_3d(n=3, seed=5, omega=0.0)
    w.v_cell = w.v_cell * 0.0
    w.v_node = w.v_node * 0.0
    P = O.Problem(w, O.default_params(w.c_cfl, detect=False))
    x = P.state.x
    top = [(c, k) for c, k in boundary_faces(w.cells)
           if np.all(np.abs(x[np.delete(w.cells[c], k), 2] - x[:, 2].max()) < 1e-12)]
    assert len(top) == 2 * 9
    Tbc = np.zeros((3, 3))
    Tbc[0, 2] = Tbc[2, 0] = 2.0e4
    P.mesh.set_loads([f[0] for f in top], [f[1] for f in top], np.ones(len(top)),
                     np.tile(_sym6(Tbc), (len(top), 1)))
    F = np.zeros_like(x)
    for c, k in top:
        for j in range(4):
            if j != k:
                F[w.cells[c, j]] += Tbc @ face_vector(x, w.cells, c, k)
    d0 = P.diagnostics()
    dt = P.initial_dt()
    s1, vs, _, _ = P.step(dt)
    d1 = P.diagnostics()
    assert np.allclose(np.array(d1["mom"]) - np.array(d0["mom"]), dt * F.sum(axis=0), rtol=1e-12,
                       atol=1e-12 * dt * np.abs(F).sum())
    work = dt * np.sum(F * vs)
    assert work > 0
    assert (d1["energy"] - d0["energy"]) == pytest.approx(work, rel=1e-9)


def _piston(U, as_wall=False):
    w = W.rotating_cube_3d(n=3, seed=6, omega=0.0)
    x = w.x
    face = [(c, k) for c, k in boundary_faces(w.cells)
            if np.all(np.abs(x[np.delete(w.cells[c], k), 0] - x[:, 0].max()) < 1e-12)]
    on = np.zeros(w.n_nodes, bool)
    for c, k in face:
        on[np.delete(w.cells[c], k)] = True
    if as_wall:
        w.nwall = np.where(on, 1, 0).astype(np.uint8)
        w.normals = np.zeros((w.n_nodes, 3, 3))
        w.normals[on, 0, 0] = 1.0
    P = O.Problem(w, O.default_params(w.c_cfl, detect=False))
    if not as_wall:
        val = np.zeros((len(face), 6))
        val[:, 0] = U
        P.mesh.set_loads([f[0] for f in face], [f[1] for f in face], np.full(len(face), 2), val)
    return w, P, face, on


def test_normal_velocity_is_met_at_every_loaded_node():
    U = -0.3
    w, P, face, on = _piston(U)
    x = P.state.x.copy()
    dt = P.initial_dt()
    _, vs, _, _ = P.step(dt)
    dvec = np.zeros_like(x)
    V = np.zeros(w.n_nodes)
    for c, k in face:
        fv = face_vector(x, w.cells, c, k)
        for j in range(4):
            if j != k:
                dvec[w.cells[c, j]] += fv
                V[w.cells[c, j]] += U * np.linalg.norm(fv)
    got = np.sum(vs * dvec, axis=1)
    assert np.allclose(got[on], V[on], rtol=1e-12, atol=1e-14)
    assert np.abs(vs[on, 0] - U).max() < 1e-12     # the face is flat: v_x = U


def test_zero_normal_velocity_is_the_slip_wall():
    _, Pv, _, on = _piston(0.0)
    _, Pw, _, _ = _piston(0.0, as_wall=True)
    dt = Pv.initial_dt()
    _, vs_v, _, _ = Pv.step(dt)
    _, vs_w, _, _ = Pw.step(dt)
    assert np.abs(vs_v[on, 0]).max() < 1e-14
    assert np.allclose(vs_v, vs_w, rtol=0, atol=1e-12 * np.abs(vs_w).max() + 1e-300)


def test_wall_takes_precedence_over_a_velocity_load():
    w, Pw, face, on = _piston(0.0, as_wall=True)
    P2 = O.Problem(w, O.default_params(w.c_cfl, detect=False))
    val = np.zeros((len(face), 6))
    val[:, 0] = -0.5
    P2.mesh.set_loads([f[0] for f in face], [f[1] for f in face], np.full(len(face), 2), val)
    dt = Pw.initial_dt()
    s1, vs1, _, _ = Pw.step(dt)
    s2, vs2, _, _ = P2.step(dt)
    assert np.array_equal(vs1, vs2) and np.array_equal(s1.v, s2.v)


def test_velocity_load_is_met_along_a_wall():
    """Hierarchy: a node on a slip wall (z = 0) and on a piston face (x = 0)
    keeps v_z = 0 and still meets the piston's normal velocity."""
    U = 0.4
    w = W.rotating_cube_3d(n=3, seed=7, omega=0.0)
    x = w.x
    bottom = np.abs(x[:, 2] - x[:, 2].min()) < 1e-12
    w.nwall = bottom.astype(np.uint8)
    w.normals = np.zeros((w.n_nodes, 3, 3))
    w.normals[bottom, 0, 2] = 1.0
    face = [(c, k) for c, k in boundary_faces(w.cells)
            if np.all(np.abs(x[np.delete(w.cells[c], k), 0] - x[:, 0].min()) < 1e-12)]
    on = np.zeros(w.n_nodes, bool)
    for c, k in face:
        on[np.delete(w.cells[c], k)] = True
    edge = on & bottom
    assert edge.sum() == 4
    P = O.Problem(w, O.default_params(w.c_cfl, detect=False))
    val = np.zeros((len(face), 6))
    val[:, 0] = -U                      # outward normal -x: v_x = U
    P.mesh.set_loads([f[0] for f in face], [f[1] for f in face], np.full(len(face), 2), val)
    dt = P.initial_dt()
    _, vs, _, _ = P.step(dt)
    assert np.abs(vs[bottom, 2]).max() <= 1e-15 * U
    assert np.abs(vs[on, 0] - U).max() <= 1e-12 * U
    # the bending field moves the edge nodes along y: they are not held
    assert np.abs(vs[edge, 1]).max() > 1e-6
