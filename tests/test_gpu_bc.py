"""Boundary loads (hl_set_boundary_loads; Section 3.8 and Appendix B,
readings R28 prescribed traction, R29 prescribed normal velocity) through
the C-ABI against the oracle: a bar driven by a piston at one end, with a
compressive traction on the other and a shear traction on its top (MOOD
re-solves loaded nodes every step), in both cascades; a 2D square; the
matching-traction equilibrium; the zero-velocity load against the slip
wall; graph capture and batches with loads; clearing; the argument checks."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

from .parity_util import FIELDS, compare_states, fmt, max_err
from .test_oracle_bc import _sym6, boundary_faces

pytestmark = pytest.mark.gpu

ONE_STEP = 1e-12
MANY = 1e-9


def _faces_on(w, axis, val):
    return [(c, k) for c, k in boundary_faces(w.cells)
            if np.all(np.abs(w.x[np.delete(w.cells[c], k), axis] - val) < 1e-12)]


def _loaded_bar(seed=3):
    """Bar [0,4]x[0,1]^2 with no walls, translating at v_x = 20: piston
    v_x = 150 on x = 0 (outward v_n = -150), normal stress -2e8 on x = 4,
    shear T13 = 5e7 on z = 1.  (A cold body at rest, e = |v| = 0, sits
    exactly on the admissibility bound eps = 0, where rounding noise of
    either implementation decides the flag; the translation keeps the
    detection well-posed.)"""
    w = W.impact_bar_3d(nx=16, ny=4, graded=False, seed=seed)
    w.nwall = np.zeros_like(w.nwall)
    w.normals = np.zeros_like(w.normals)
    w.v_cell = w.v_cell * 0.0 + np.array([20.0, 0.0, 0.0])
    w.v_node = w.v_node * 0.0 + np.array([20.0, 0.0, 0.0])
    left, right, top = _faces_on(w, 0, 0.0), _faces_on(w, 0, 4.0), _faces_on(w, 2, 1.0)
    faces = left + right + top
    kind = np.array([2] * len(left) + [1] * (len(right) + len(top)), np.uint8)
    val = np.zeros((len(faces), 6))
    val[:len(left), 0] = -150.0
    val[len(left):len(left) + len(right), 0] = -2e8
    val[len(left) + len(right):, 4] = 5e7
    return w, (np.array([f[0] for f in faces], np.int32), np.array([f[1] for f in faces], np.uint8), kind, val)


def _loaded_square():
    """Unit square with no walls: v_n = -0.02 on x = 0, traction T11 = -0.05
    on x = 1 and T12 = 0.03 on y = 1."""
    w = W.plane_wave_2d(n=12, amp=0.01, seed=8)
    w.nwall = np.zeros_like(w.nwall)
    w.normals = np.zeros_like(w.normals)
    left, right, top = _faces_on(w, 0, 0.0), _faces_on(w, 0, 1.0), _faces_on(w, 1, 1.0)
    faces = left + right + top
    kind = np.array([2] * len(left) + [1] * (len(right) + len(top)), np.uint8)
    val = np.zeros((len(faces), 6))
    val[:len(left), 0] = -0.02
    val[len(left):len(left) + len(right), 0] = -0.05
    val[len(left) + len(right):, 3] = 0.03
    return w, (np.array([f[0] for f in faces], np.int32), np.array([f[1] for f in faces], np.uint8), kind, val)


def _pair(w, loads, cascade=2):
    ctx = H.from_workload(w, params=H.default_params(w.dim, c_cfl=w.c_cfl, cascade=cascade))
    prob = O.Problem(w, O.default_params(w.c_cfl, cascade=cascade))
    ctx.set_boundary_loads(*loads)
    prob.mesh.set_loads(*loads)
    return ctx, prob


@pytest.mark.parametrize("cascade", [2, 3])
def test_loaded_bar_parity(cascade):
    w, loads = _loaded_bar()
    ctx, prob = _pair(w, loads, cascade)
    dt = prob.initial_dt()
    ctx.step(dt)
    s1, vs, mk, oi = prob.step(dt)
    e = compare_states(ctx, s1, vs)
    print(f"[bc bar c{cascade}] step 1: {fmt(e)} p0 {oi.n_p0} lim {oi.n_lim}", flush=True)
    assert np.array_equal(ctx.query("order"), mk)
    assert oi.n_p0 > 0
    assert max_err(e) <= ONE_STEP, fmt(e)
    dt = oi.dt_next
    flips = passes = 0
    for _ in range(29):
        info = ctx.step(dt)
        _, _, mk, oi = prob.step(dt)
        flips += int(not np.array_equal(ctx.query("order"), mk))
        passes = max(passes, oi.mood_iters)
        assert info["mood_iters"] == oi.mood_iters
        dt = oi.dt_next
    e = compare_states(ctx, prob.state)
    print(f"[bc bar c{cascade}] 30 steps: {fmt(e)} mask-differing steps {flips} max passes {passes}", flush=True)
    assert flips == 0 and passes >= 3
    assert max_err(e) <= MANY, fmt(e)


def test_loaded_square_parity_2d():
    w, loads = _loaded_square()
    ctx, prob = _pair(w, loads)
    dt = prob.initial_dt()
    for n in range(20):
        ctx.step(dt)
        s1, vs, mk, oi = prob.step(dt)
        assert np.array_equal(ctx.query("order"), mk)
        if n == 0:
            e = compare_states(ctx, s1, vs)
            assert max_err(e) <= ONE_STEP, fmt(e)
        dt = oi.dt_next
    e = compare_states(ctx, prob.state)
    print(f"[bc square] 20 steps: {fmt(e)}", flush=True)
    assert max_err(e) <= MANY, fmt(e)


def test_matching_traction_keeps_a_stressed_cube_at_rest():
    w = W.rotating_cube_3d(n=4, seed=4, omega=0.0)
    J = 0.97
    rho0, mu, K = w.rho0[0], w.mu[0], w.lam[0] + 2.0 * w.mu[0] / 3.0
    B3 = np.eye(3) * J ** (2.0 / 3.0)
    T, p, a, _ = O.point_stress(rho0, mu, K, J / rho0, B3)
    ctx = H.from_workload(w, params=H.default_params(3, detect=False, c_cfl=w.c_cfl))
    st = ctx.state()
    st["tau"][:] = J / rho0
    st["v"][:] = 0.0
    st["vhat"][:] = 0.0
    st["e"][:] = 0.0
    st["B"][:] = 0.0
    st["B"][:, :3] = J ** (2.0 / 3.0)
    ctx.set_state(st)
    faces = boundary_faces(w.cells)
    dt = 0.5 * ctx.compute_dt()
    ctx.step(dt)
    free = np.abs(ctx.query("vstar")).max()
    ctx.set_state(st)
    ctx.set_boundary_loads(np.array([f[0] for f in faces], np.int32), np.array([f[1] for f in faces], np.uint8),
                           np.ones(len(faces), np.uint8), np.tile(_sym6(T), (len(faces), 1)))
    ctx.step(dt)
    held = np.abs(ctx.query("vstar")).max()
    scale = abs(p) / (rho0 * a)
    print(f"[bc equilibrium] free {free:.3e} held {held:.3e} scale {scale:.3e}", flush=True)
    assert free > 1e-3 * scale and held <= 1e-12 * scale


def test_zero_normal_velocity_is_the_slip_wall():
    w = W.rotating_cube_3d(n=4, seed=6, omega=1.0)
    face = _faces_on(w, 0, 1.0)
    on = np.zeros(w.n_nodes, bool)
    for c, k in face:
        on[np.delete(w.cells[c], k)] = True
    loaded = H.from_workload(w)
    loaded.set_boundary_loads(np.array([f[0] for f in face], np.int32), np.array([f[1] for f in face], np.uint8),
                              np.full(len(face), 2, np.uint8), np.zeros((len(face), 6)))
    ww = W.rotating_cube_3d(n=4, seed=6, omega=1.0)
    ww.nwall = np.where(on, 1, 0).astype(np.uint8)
    ww.normals = np.zeros((w.n_nodes, 3, 3))
    ww.normals[on, 0, 0] = 1.0
    ww.v_node = ww.v_node.copy()
    ww.v_node[on, 0] = 0.0
    wall = H.from_workload(ww)
    loaded.upload_field("vhat", wall.query("vhat"))
    dt = 0.5 * wall.compute_dt()
    for _ in range(5):
        loaded.step(dt)
        wall.step(dt)
        vl, vw = loaded.query("vstar"), wall.query("vstar")
        assert np.abs(vl[on, 0]).max() < 1e-14 * np.abs(vw).max()
        assert np.allclose(vl, vw, rtol=0, atol=1e-12 * np.abs(vw).max())


def test_velocity_load_along_a_wall_parity():
    """BC hierarchy: a piston face (x = 0) meets a slip floor (z = 0); the
    edge nodes keep v_z = 0 and meet the piston velocity."""
    U = 0.4
    w = W.rotating_cube_3d(n=4, seed=7, omega=0.5)
    bottom = np.abs(w.x[:, 2]) < 1e-12
    w.nwall = bottom.astype(np.uint8)
    w.normals = np.zeros((w.n_nodes, 3, 3))
    w.normals[bottom, 0, 2] = 1.0
    face = _faces_on(w, 0, 0.0)
    on = np.zeros(w.n_nodes, bool)
    for c, k in face:
        on[np.delete(w.cells[c], k)] = True
    val = np.zeros((len(face), 6))
    val[:, 0] = -U
    loads = (np.array([f[0] for f in face], np.int32), np.array([f[1] for f in face], np.uint8),
             np.full(len(face), 2, np.uint8), val)
    ctx, prob = _pair(w, loads)
    dt = prob.initial_dt()
    for n in range(10):
        ctx.step(dt)
        s1, vs, mk, oi = prob.step(dt)
        assert np.array_equal(ctx.query("order"), mk)
        g = ctx.query("vstar")
        if n == 0:
            e = compare_states(ctx, s1, vs)
            assert max_err(e) <= ONE_STEP, fmt(e)
        assert np.abs(g[bottom, 2]).max() <= 1e-15 * U
        assert np.abs(g[on & bottom, 0] - U).max() <= 1e-12 * U
        dt = oi.dt_next
    e = compare_states(ctx, prob.state)
    print(f"[bc wall+piston] 10 steps: {fmt(e)}", flush=True)
    assert max_err(e) <= MANY, fmt(e)


def _same(a, b):
    sa, sb = a.state(), b.state()
    for f in FIELDS:
        if not np.array_equal(sa[f], sb[f]):
            return f
    return None if np.array_equal(a.query("order"), b.query("order")) else "order"


def test_graph_with_loads_equals_eager():
    w, loads = _loaded_bar(seed=5)
    eager, graph = H.from_workload(w), H.from_workload(w)
    graph.use_graph(True, 6)
    for c in (eager, graph):
        c.set_boundary_loads(*loads)
        c.compute_dt()
    for k in range(8):
        eager.step(0.0)
        graph.step(0.0)
        assert _same(eager, graph) is None, k
    # new loads after capture: the graph is rebuilt with them
    cell, face, kind, val = loads
    val = val * 0.5
    for c in (eager, graph):
        c.set_boundary_loads(cell, face, kind, val)
    for k in range(4):
        eager.step(0.0)
        graph.step(0.0)
        assert _same(eager, graph) is None, ("reloaded", k)


def test_batch_with_loads_equals_single_meshes():
    wb, loads = _loaded_bar(seed=7)
    wc = W.rotating_cube_3d(n=3, seed=2)
    bctx = H.from_workloads([wc, wb])
    cell, face, kind, val = loads
    bctx.set_boundary_loads(cell + wc.n_cells, face, kind, val)
    sc, sb = H.from_workload(wc), H.from_workload(wb)
    sb.set_boundary_loads(*loads)
    for c in (bctx, sc, sb):
        c.compute_dt()
    for _ in range(6):
        bctx.step_batch(None)
        sc.step(0.0)
        sb.step(0.0)
    st = bctx.state()
    no, co = bctx.node_offsets, bctx.cell_offsets
    for m, s in enumerate((sc, sb)):
        ss = s.state()
        for f in ("x", "vhat"):
            assert np.array_equal(st[f][no[m]:no[m + 1]], ss[f]), (m, f)
        for f in ("tau", "v", "e", "B"):
            assert np.array_equal(st[f][co[m]:co[m + 1]], ss[f]), (m, f)


def test_clearing_loads_and_argument_checks():
    w, loads = _loaded_bar(seed=9)
    plain, cleared = H.from_workload(w), H.from_workload(w)
    cleared.set_boundary_loads(*loads)
    cleared.set_boundary_loads()
    dt = plain.compute_dt()
    for _ in range(3):
        plain.step(dt)
        cleared.step(dt)
    assert _same(plain, cleared) is None
    cell, face, kind, val = loads
    bad = [(cell + w.n_cells, face, kind, val), (cell, face + 4, kind, val), (cell, face, kind * 0 + 3, val)]
    nan = val.copy()
    nan[0, 0] = np.nan
    bad.append((cell, face, kind, nan))
    for args in bad:
        with pytest.raises(H.HyperLagError):
            plain.set_boundary_loads(*args)
    with pytest.raises(ValueError):
        plain.set_boundary_loads(cell, face, kind, val[:, :3])
    plain.set_boundary_loads(*loads)
    with pytest.raises(H.HyperLagError):
        plain.forward_record(2, 1)
    # a new mesh drops the loads: its step equals a fresh context's
    plain.upload_mesh(w.dim, w.x, w.cells, w.nwall, w.normals)
    H.init_from_workloads(plain, [w])
    fresh = H.from_workload(w)
    plain.step(dt)
    fresh.step(dt)
    assert _same(plain, fresh) is None
