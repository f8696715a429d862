"""Pins of the oracle's detection, time-step control, singular stencils and
involution monitors against values the paper's rules fix by hand.

Each case is built so that a plausible slip in the oracle changes the
expected answer:
  - the relaxed DMP (Section 3.5, eq. RDMP): delta = max(delta0,
    delta1 (M - m)) on rho = 1/tau over the cell and every cell sharing a
    node with it;
  - physical admissibility (eq. PAD, reading R16): non-finite values,
    tau > 0, det B > 0, eps >= -tol (|e| + |v|^2/2), and p + p_inf > 0 for
    the stiffened gas (R31);
  - the time step (Section 3.6, eqs. CFL, CFL2; R20): C_v dt min V1/|dV|,
    (1 + C_i) dt, acoustic only at the first step;
  - the least-squares rule for stencils that cannot fix a gradient (R8);
  - the GCL with Simpson-averaged corner vectors and the det B monitor
    (eq. test_detB_rho, R19);
  - the count of cells the MOOD loop recomputes (R18).
Expected values are numbers chosen by hand, closed forms of the special
case, or sets counted here from the connectivity alone.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import workloads as W


def _quiet_candidate(prob, rho):
    """A candidate at rest (v = 0, B = I, e > 0) with density rho per cell."""
    nc, d = prob.mesh.nc, prob.dim
    B = np.zeros((nc, prob.mesh.nB))
    B[:, :d] = 1.0   # diagonal components come first: (11, 22[, 33], ...)
    st = prob.state.copy()
    st.tau = 1.0 / np.asarray(rho, dtype=np.float64)
    st.v = np.zeros((nc, d))
    st.e = np.full(nc, 1.0)
    st.B = B
    return st


def _node_neighbours(cells):
    """For every cell, the set of cells sharing at least one node with it."""
    by_node = {}
    for c, nodes in enumerate(cells):
        for p in nodes:
            by_node.setdefault(int(p), []).append(c)
    return [set(j for p in nodes for j in by_node[int(p)]) for nodes in cells]


def _mesh2d():
    w = W.plane_wave_2d(n=6)
    return w, O.Problem(w, O.default_params(w.c_cfl))


def _interior_cell(w):
    x = w.x[w.cells].mean(axis=1)
    return int(np.argmin(np.abs(x - 0.5).sum(axis=1)))


# ------------------------------------------------------------- RDMP

def test_rdmp_absolute_tolerance_delta0():
    """Uniform rho^n = 1000: M - m = 0, so delta = delta0 = 1e-4 (absolute,
    kg/m^3).  A candidate rho within 0.9e-4 of 1000 passes, 1.1e-4 away is
    flagged, on either side."""
    w, P = _mesh2d()
    nc = P.mesh.nc
    st0 = P.state.copy()
    st0.tau = np.full(nc, 1e-3)
    c = _interior_cell(w)
    for drho, want in ((0.9e-4, 0), (1.1e-4, 2), (-0.9e-4, 0), (-1.1e-4, 2)):
        rho = np.full(nc, 1000.0)
        rho[c] = 1000.0 + drho
        code = P.detect(_quiet_candidate(P, rho), state=st0)
        assert code[c] == want, (drho, code[c])
        others = np.delete(code, c)
        assert not others.any()


def test_rdmp_relative_tolerance_delta1_on_density():
    """rho^n in [1000, 1002] around the cell: delta = delta1 (M - m) =
    2e-3 > delta0.  rho = 1002 + 1.9e-3 passes, 1002 + 2.1e-3 fails, and
    1000 - 2.1e-3 fails.  A tolerance of delta1 * M (about 1) or bounds
    taken on tau instead of rho would pass all three."""
    w, P = _mesh2d()
    nc = P.mesh.nc
    c = _interior_cell(w)
    nb = sorted(_node_neighbours(w.cells)[c] - {c})
    rho0 = np.full(nc, 1000.0)
    rho0[nb[0]] = 1002.0
    st0 = P.state.copy()
    st0.tau = 1.0 / rho0
    for r1, want in ((1002.0 + 1.9e-3, 0), (1002.0 + 2.1e-3, 2), (1000.0 - 2.1e-3, 2),
                     (1000.0 - 1.9e-3, 0)):
        rho = rho0.copy()
        rho[c] = r1
        code = P.detect(_quiet_candidate(P, rho), state=st0)
        assert code[c] == want, (r1, code[c])


def test_rdmp_neighbourhood_is_every_cell_sharing_a_node():
    """The bounds run over the cell and every cell that shares a node with
    it (reading R8; the paper's "von Neumann neighbourhood used to
    reconstruct"): a cell touching c at one vertex only widens c's bounds,
    a cell touching none does not."""
    w, P = _mesh2d()
    nc = P.mesh.nc
    c = _interior_cell(w)
    share = [len(set(w.cells[c]) & set(w.cells[j])) for j in range(nc)]
    vertex_only = [j for j in range(nc) if share[j] == 1]
    far = [j for j in range(nc) if share[j] == 0]
    assert vertex_only and far
    st0 = P.state.copy()
    # a vertex-only neighbour at 1010: c may rise to 1010 (+ delta1 * 10)
    rho0 = np.full(nc, 1000.0)
    rho0[vertex_only[0]] = 1010.0
    st0.tau = 1.0 / rho0
    rho = rho0.copy()
    rho[c] = 1010.0
    assert P.detect(_quiet_candidate(P, rho), state=st0)[c] == 0
    # a cell sharing no node at 1010: c's bounds stay [1000, 1000]
    rho0 = np.full(nc, 1000.0)
    rho0[far[-1]] = 1010.0
    st0.tau = 1.0 / rho0
    rho = rho0.copy()
    rho[c] = 1005.0
    assert P.detect(_quiet_candidate(P, rho), state=st0)[c] == 2


def test_rdmp_not_applied_to_first_order_cells():
    """First-order cells are accepted as the parachute (Section 3.5)."""
    w, P = _mesh2d()
    nc = P.mesh.nc
    c = _interior_cell(w)
    rho = np.full(nc, 1000.0)
    rho[c] = 1100.0
    st0 = P.state.copy()
    st0.tau = np.full(nc, 1e-3)
    mask = np.zeros(nc, np.uint8)
    assert P.detect(_quiet_candidate(P, rho), state=st0, mask=mask)[c] == 2
    mask[c] = 2
    assert P.detect(_quiet_candidate(P, rho), state=st0, mask=mask)[c] == 0


# -------------------------------------------------------------- PAD

def _pad_case(dim):
    if dim == 2:
        w = W.plane_wave_2d(n=4)
    else:
        w = W.impact_bar_3d(nx=4, ny=2, graded=False)
    P = O.Problem(w, O.default_params(w.c_cfl))
    st0 = P.state.copy()
    return w, P, st0


@pytest.mark.parametrize("dim", [2, 3])
def test_pad_non_finite_and_volume(dim):
    """Any non-finite value, and tau <= 0, make a candidate inadmissible
    (code 1).  tau = 0 exactly is inadmissible (tau > 0 is strict); a tiny
    positive tau is admissible and only the relaxed DMP rejects it."""
    w, P, st0 = _pad_case(dim)
    c = 1
    base = _quiet_candidate(P, 1.0 / st0.tau)
    assert not P.detect(base, state=st0).any()
    for field, idx, val in (("tau", (c,), np.nan), ("e", (c,), np.inf), ("v", (c, 0), np.nan),
                            ("v", (c, dim - 1), -np.inf), ("B", (c, 0), np.nan), ("B", (c, -1), np.inf)):
        cand = base.copy()
        getattr(cand, field)[idx] = val
        code = P.detect(cand, state=st0)
        assert code[c] == 1, (field, idx, val)
    for tau1, want in ((0.0, 1), (-st0.tau[c], 1), (1e-300, 2)):
        cand = base.copy()
        cand.tau[c] = tau1
        assert P.detect(cand, state=st0)[c] == want, tau1


@pytest.mark.parametrize("dim", [2, 3])
def test_pad_det_b(dim):
    """det B <= 0 is inadmissible (B is a left Cauchy-Green tensor); a
    positive diagonal does not make det B positive."""
    w, P, st0 = _pad_case(dim)
    c = 2
    base = _quiet_candidate(P, 1.0 / st0.tau)
    # 11, 22, 12 in 2D; 11, 22, 33, 12, 13, 23 in 3D
    i12 = 2 if dim == 2 else 3
    for b11, b22, b12, want in ((1.0, 1.0, 1.0, 1),        # det = 0
                                (1.0, 1.0, 2.0, 1),        # det < 0, diagonal > 0
                                (1.0, 1.0, 1.0 - 1e-9, 0),  # det > 0, tiny
                                (2.0, 0.5, 0.0, 0)):
        cand = base.copy()
        cand.B[c, 0], cand.B[c, 1], cand.B[c, i12] = b11, b22, b12
        assert P.detect(cand, state=st0)[c] == want, (b11, b22, b12)


@pytest.mark.parametrize("dim", [2, 3])
def test_pad_internal_energy_tolerance(dim):
    """eps = e - |v|^2/2 is troubled below -1e-12 (|e| + |v|^2/2) (R16):
    with |v| = 150 m/s the bound is about 2.25e-8 J/kg, so 0.9 of it passes
    and 1.1 of it fails; an absolute 1e-12 or a |v|^2 kinetic term would
    flag both."""
    w, P, st0 = _pad_case(dim)
    c = 3
    v = np.zeros(dim)
    v[0] = 150.0
    k = 0.5 * 150.0 ** 2
    for frac, want in ((0.9, 0), (1.1, 1), (0.0, 0)):
        cand = _quiet_candidate(P, 1.0 / st0.tau)
        # solve e - k = -frac * 1e-12 (|e| + k) for e
        e = k * (1.0 - frac * 1e-12) / (1.0 + frac * 1e-12)
        cand.v[c] = v
        cand.e[c] = e
        assert P.detect(cand, state=st0)[c] == want, frac


def test_pad_stiffened_gas_hyperbolicity():
    """Stiffened gas (R31): a state with p + p_inf <= 0 is troubled.  At
    B = I the shear energy vanishes and p + p_inf = (gamma - 1)(eps / tau -
    p_inf), so eps = p_inf tau (1 -+ 1e-6) sits just on either side."""
    w = W.plane_wave_2d(n=4)
    prm = O.default_params(w.c_cfl, eos=1, sg_gamma=2.2, sg_pinf=1e6)
    P = O.Problem(w, prm)
    st0 = P.state.copy()
    c = 5
    for f, want in ((1.0 - 1e-6, 1), (1.0 + 1e-6, 0)):
        cand = _quiet_candidate(P, 1.0 / st0.tau)
        cand.e = np.array(P.state.e, copy=True)
        cand.e[c] = 1e6 * cand.tau[c] * f
        assert P.detect(cand, state=st0)[c] == want, f


# ------------------------------------------------------- time step

def _dilated(P, s):
    """The held state with every node at (1 + s) x: V1 = (1 + s)^d V0."""
    st = P.state.copy()
    st.x = st.x * (1.0 + s)
    st.tau = st.tau * (1.0 + s) ** P.dim
    return st


@pytest.mark.parametrize("dim", [2, 3])
def test_time_step_volume_bound_closed_form(dim):
    """A uniform dilation by 1 + s changes every cell volume by the same
    factor, so dt_vol = C_v dt V1 / |V1 - V0| = C_v dt (1+s)^d /
    ((1+s)^d - 1) (eq. CFL2, reading R20); at s = 0.2 it binds below the
    growth bound 1.1 dt and far below the acoustic bound."""
    w, P, _ = _pad_case(dim)
    V0 = P.m * P.state.tau
    acoustic = P.initial_dt()
    dt_prev = 1e-3 * acoustic
    f = 1.2 ** dim
    info = P.time_step(_dilated(P, 0.2), dt_prev, V0)
    want = 0.2 * dt_prev * f / (f - 1.0)
    assert info.dt_volume == pytest.approx(want, rel=1e-12)
    assert info.dt_next == pytest.approx(want, rel=1e-12)
    assert want < 1.1 * dt_prev < info.dt_acoustic


@pytest.mark.parametrize("dim", [2, 3])
def test_time_step_growth_bound(dim):
    """No volume change (cells with dV = 0 are skipped) and a small previous
    step: dt_next = (1 + C_i) dt = 1.1 dt, the growth bound of eq. CFL2 read
    as (1 + C_i) dt (R20), not C_i dt."""
    w, P, _ = _pad_case(dim)
    V0 = P.m * P.state.tau
    acoustic = P.initial_dt()
    dt_prev = 1e-3 * acoustic
    info = P.time_step(P.state, dt_prev, V0)
    assert math.isinf(info.dt_volume)
    assert info.dt_next == pytest.approx(1.1 * dt_prev, rel=1e-15)
    # a large previous step: the acoustic bound binds
    info = P.time_step(P.state, 10.0 * acoustic, V0)
    assert info.dt_next == info.dt_acoustic == pytest.approx(acoustic, rel=1e-15)


def test_time_step_first_step_is_acoustic_only():
    """The first step has no previous dt: only the acoustic bound applies,
    even when the volumes change."""
    w, P, _ = _pad_case(3)
    info = P.time_step(_dilated(P, 0.1), 0.0, P.m * P.state.tau)
    assert math.isinf(info.dt_volume)
    assert info.dt_next == info.dt_acoustic


# ------------------------------------------------ singular stencils

def _lsq_of(dim, x, cells, fields):
    w = W.plane_wave_2d(n=2) if dim == 2 else W.impact_bar_3d(nx=1, ny=1, graded=False)
    nc = len(cells)
    import copy
    g = copy.copy(w)
    g.x = np.asarray(x, np.float64)
    g.cells = np.asarray(cells, np.int32)
    g.nwall = np.zeros(len(x), np.uint8)
    g.normals = np.zeros((len(x), dim, dim))
    g.rho0 = np.full(nc, 1000.0)
    g.mu = np.full(nc, 1e6)
    g.lam = np.full(nc, 2e6)
    g.v_cell = np.zeros((nc, dim))
    g.v_node = np.zeros((len(x), dim))
    P = O.Problem(g)
    st = P.state.copy()
    st.tau = np.asarray(fields, np.float64)
    return P.lsq(st)


def test_lsq_stencils_that_cannot_fix_a_gradient_give_zero():
    """Reading R8: a stencil with fewer than d neighbour visits, or whose
    normal matrix is singular, gives a zero gradient (finite, no solve of a
    singular system)."""
    # a lone tetrahedron: no neighbours
    g = _lsq_of(3, [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], [[0, 1, 2, 3]], [1e-3])
    assert np.all(g == 0.0)
    # two tetrahedra sharing one node: one visit each (< 3)
    x = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1]]
    g = _lsq_of(3, x, [[0, 1, 2, 3], [0, 4, 6, 5]], [1e-3, 2e-3])
    assert np.all(g == 0.0)
    # two triangles sharing an edge: two visits at the same offset, rank 1
    g = _lsq_of(2, [[0, 0], [1, 0], [0, 1], [1, 1]], [[0, 1, 2], [1, 3, 2]], [1e-3, 2e-3])
    assert np.all(np.isfinite(g)) and np.all(g == 0.0)
    # three triangles around a node with independent offsets: a gradient
    x = [[0, 0], [1, 0], [0, 1], [-1, 0.2], [0.3, -1]]
    g = _lsq_of(2, x, [[0, 1, 2], [0, 2, 3], [0, 4, 1]], [1e-3, 2e-3, 3e-3])
    assert np.abs(g[0, 0]).max() > 0.0


# --------------------------------------------- involution monitors

def test_gcl_defect_is_roundoff_with_simpson_corner_vectors():
    """The Simpson average of the corner vectors over a step makes the
    discrete GCL V1 - V0 = dt sum_p Cbar_p . v*_p exact (eq. GCL): on a
    step with large motion the reported defect is at roundoff, while the
    corner vectors of t^n alone miss it by orders of magnitude (computed
    here with numpy volumes)."""
    w = W.rotating_cube_3d(n=3, omega=50.0)
    P = O.Problem(w, O.default_params(w.c_cfl, detect=False))
    dt = 4.0 * P.initial_dt()
    st0 = P.state.copy()
    s1, vs, _, info = P.step(dt)
    assert info.gcl_defect < 1e-13
    # the same flux with t^n corner vectors only: O(dt^2) off
    X0 = st0.x[w.cells]
    X1 = s1.x[w.cells]
    V0 = np.linalg.det(X0[:, 1:] - X0[:, :1]) / 6.0
    V1 = np.linalg.det(X1[:, 1:] - X1[:, :1]) / 6.0
    flux0 = np.zeros(len(w.cells))
    for c, nodes in enumerate(w.cells):
        for k in range(4):
            h = 1e-7
            for i in range(3):
                Xp = X0[c].copy()
                Xm = X0[c].copy()
                Xp[k, i] += h
                Xm[k, i] -= h
                dV = (np.linalg.det(Xp[1:] - Xp[0]) - np.linalg.det(Xm[1:] - Xm[0])) / 12.0 / h
                flux0[c] += dV * vs[nodes[k], i]
    assert np.max(np.abs(V1 - V0 - dt * flux0) / V0) > 1e3 * max(info.gcl_defect, 1e-16)


def test_detb_monitor():
    """|sqrt(det B) - J| with J = rho0 tau (eq. test_detB_rho read with
    J = rho0 / rho, R19), counted where it reaches L_c^3.  A state with
    J = 1 and sqrt(det B) = 1.03: the defect is 0.03; the cells' in-sphere
    diameter is about 0.2, so L_c^3 (0.008) < 0.03 < L_c^2 (0.04) and every
    cell is counted (L_c or L_c^2 as the bound would count none)."""
    w = W.rotating_cube_3d(n=2, jitter=0.0)   # cubes of side 1/2: L_c = 0.2071
    P = O.Problem(w, O.default_params(w.c_cfl, detect=False))
    st = P.state.copy()
    st.B[:, 0] = 1.03 ** 2
    dt = 1e-9 * P.initial_dt()
    _, _, _, info = P.step(dt, state=st)
    assert info.detB_defect == pytest.approx(0.03, rel=1e-6)
    assert info.n_detB == P.mesh.nc
    Lc = O.cell_geometry(w.x[w.cells[0]])["Lc"]
    assert Lc ** 3 < 0.03 < Lc ** 2


def test_recompute_count_of_a_single_mood_pass():
    """After one MOOD iteration (mood_iters == 2) the loop recomputes the
    cells that share a node with a flagged cell (R18); they are counted
    here from the connectivity and the final mask alone."""
    w = W.impact_bar_3d(nx=16, ny=4, graded=False)
    P = O.Problem(w)
    dt = P.initial_dt()
    seen = 0
    nb = _node_neighbours(w.cells)
    for _ in range(6):
        _, _, mask, info = P.step(dt)
        dt = info.dt_next
        if info.mood_iters == 2:
            flagged = np.nonzero(mask == 2)[0]
            touched = set()
            for c in flagged:
                touched |= nb[c]
            assert info.n_recomp == len(touched)
            seen += 1
        elif info.mood_iters > 2:
            assert info.n_recomp > 0
        else:
            assert info.n_recomp == 0
    assert seen >= 1
