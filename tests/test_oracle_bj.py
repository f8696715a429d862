"""Pins of the oracle's three-level cascade P1 -> P1 with the Barth-Jespersen
limiter -> P0 (Section 3.5, the second scheme of the cascade; Section 3.7).

The limiter is pinned by the properties that define it rather than by its
formula: the limited linear reconstruction stays inside the min/max of the
cell values over {c} and its stencil at every vertex; the limiting factor
is the largest one in [0, 1] that does so (below 1 some vertex sits on a
bound); a linear field is not limited inside the mesh; a local extremum
loses its slope.  The cascade is pinned by conservation, the GCL identity
and the fixpoint of the MOOD loop with three levels.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import workloads as W

from .test_oracle_pins import _gcl_defect


def _W(P, s):
    """Reconstructed scalars per cell: tau, v, stored B components."""
    return np.concatenate([s.tau[:, None], s.v, s.B], axis=1)


def _stencil_bounds(cells, Wc):
    """min / max of each scalar over {c} and every cell sharing a node."""
    nn = cells.max() + 1
    lo_n = np.full((nn, Wc.shape[1]), np.inf)
    hi_n = np.full((nn, Wc.shape[1]), -np.inf)
    for k in range(cells.shape[1]):
        np.minimum.at(lo_n, cells[:, k], Wc)
        np.maximum.at(hi_n, cells[:, k], Wc)
    return lo_n[cells].min(axis=1), hi_n[cells].max(axis=1)


def _perturbed(w, seed, jump=False):
    """A general state: smooth fields plus noise, optionally a jump."""
    P = O.Problem(w)
    s = P.state.copy()
    rng = np.random.default_rng(seed)
    xc = s.x[w.cells].mean(axis=1)
    d = w.dim
    s.tau = s.tau * (1.0 + 0.05 * np.sin(3.0 * xc[:, 0]) + 0.01 * rng.standard_normal(w.n_cells))
    s.v = s.v + 0.1 * np.cos(2.0 * xc[:, :d]) + 0.02 * rng.standard_normal((w.n_cells, d))
    s.B = s.B + 0.02 * rng.standard_normal(s.B.shape)
    if jump:
        s.tau = np.where(xc[:, 0] > 0.5, s.tau * 1.3, s.tau)
    return P, s


CASES = {
    "tri": lambda: W.plane_wave_2d(n=10, amp=0.0, seed=3),
    "tet": lambda: W.rotating_cube_3d(n=4, seed=3),
}


def _vertex_values(w, s, Wc, g):
    xc = s.x[w.cells].mean(axis=1)
    dl = s.x[w.cells] - xc[:, None, :]              # [nc, d+1, d]
    return Wc[:, None, :] + np.einsum("cwi,cki->ckw", g, dl)   # [nc, d+1, nW]


@pytest.mark.parametrize("jump", [False, True])
@pytest.mark.parametrize("case", list(CASES))
def test_limited_reconstruction_stays_in_stencil_bounds(case, jump):
    w = CASES[case]()
    P, s = _perturbed(w, 7, jump)
    Wc = _W(P, s)
    lo, hi = _stencil_bounds(w.cells, Wc)
    g = P.lsq(s)
    gl = P.bj(s)
    vals = _vertex_values(w, s, Wc, gl)
    scale = np.abs(Wc).max(axis=0)
    tol = 1e-13 * scale
    assert np.all(vals >= lo[:, None, :] - tol)
    assert np.all(vals <= hi[:, None, :] + tol)
    # the unlimited reconstruction does leave the bounds, so the test bites
    raw = _vertex_values(w, s, Wc, g)
    assert np.any(raw > hi[:, None, :] + tol) or np.any(raw < lo[:, None, :] - tol)


@pytest.mark.parametrize("case", list(CASES))
def test_limiting_factor_is_the_largest_admissible_one(case):
    w = CASES[case]()
    P, s = _perturbed(w, 8, jump=True)
    Wc = _W(P, s)
    lo, hi = _stencil_bounds(w.cells, Wc)
    g = P.lsq(s)
    gl = P.bj(s)
    # gl = phi g with phi in [0, 1], one phi per cell and scalar
    gn = np.linalg.norm(g, axis=2)
    ok = gn > 1e-300
    phi = np.where(ok, np.einsum("cwi,cwi->cw", gl, g) / np.where(ok, gn ** 2, 1.0), 1.0)
    assert np.all(phi >= -1e-15) and np.all(phi <= 1.0 + 1e-15)
    assert np.allclose(gl, phi[:, :, None] * g, rtol=0, atol=1e-14 * np.abs(g).max())
    # below 1, a vertex value lies on a bound: a larger factor would leave it
    vals = _vertex_values(w, s, Wc, gl)
    gap = np.minimum(np.abs(vals - hi[:, None, :]), np.abs(vals - lo[:, None, :])).min(axis=1)
    limited = ok & (phi < 1.0 - 1e-12)
    assert limited.sum() > 0
    scale = np.abs(Wc).max(axis=0)[None, :] * np.ones_like(gap)
    assert np.all(gap[limited] <= 1e-12 * scale[limited])
    assert (phi[ok] == 0.0).any() and (phi[ok] == 1.0).any()


@pytest.mark.parametrize("case", list(CASES))
def test_linear_field_is_not_limited_inside(case):
    """Every interior vertex is surrounded by the centroids of its cells,
    so an affine field's vertex values stay inside the stencil range."""
    w = CASES[case]()
    P = O.Problem(w)
    s = P.state.copy()
    xc = s.x[w.cells].mean(axis=1)
    a = np.arange(1, w.dim + 1, dtype=float)
    s.tau = 1.0 + 0.1 * xc @ a
    s.v = 0.2 + xc @ np.ones((w.dim, w.dim)) * 0.3
    s.B = 1.0 + 0.05 * (xc @ np.ones((w.dim, s.B.shape[1])))
    g = P.lsq(s)
    gl = P.bj(s)
    node_boundary = np.zeros(s.x.shape[0], bool)
    for i in range(w.dim):
        node_boundary |= (np.abs(s.x[:, i] - s.x[:, i].min()) < 1e-12) | \
                         (np.abs(s.x[:, i] - s.x[:, i].max()) < 1e-12)
    inner = ~node_boundary[w.cells].any(axis=1)
    assert inner.sum() > 0
    assert np.array_equal(gl[inner], g[inner])


def test_local_extremum_loses_its_slope():
    w = CASES["tet"]()
    P, s = _perturbed(w, 9)
    c = 60
    s.tau[c] = s.tau.max() * 1.5       # a strict local maximum of tau
    g = P.lsq(s)
    gl = P.bj(s)
    assert np.abs(g[c, 0]).max() > 0
    assert np.all(gl[c, 0] == 0.0)


def _bar():
    return W.impact_bar_3d(nx=16, ny=4, graded=True, seed=11)


def test_three_level_cascade_conserves_and_keeps_the_gcl():
    """Sec. 3.3 and reading R12 with the three-level cascade: mass, total
    energy and the GCL identity; limited cells appear."""
    w = _bar()
    P = O.Problem(w, O.default_params(w.c_cfl, cascade=3))
    d0 = P.diagnostics()
    dt = P.initial_dt()
    n_lim = 0
    for _ in range(5):
        x0 = P.state.x.copy()
        s1, vstar, mk, info = P.step(dt)
        assert _gcl_defect(w, x0, s1.x, vstar, dt, None) < 1e-12
        assert info.n_lim == (mk == 1).sum() and info.n_p0 == (mk == 2).sum()
        n_lim += info.n_lim
        dt = info.dt_next
    assert n_lim > 0
    d1 = P.diagnostics()
    assert d1["mass"] == d0["mass"]
    assert d1["energy"] == pytest.approx(d0["energy"], rel=1e-13)


def test_three_level_fixpoint_replays_bitwise():
    """Sec. 3.7: the loop ends on a mask whose replay reproduces the step
    bitwise, with cells at both lower levels of the cascade."""
    w = _bar()
    P = O.Problem(w, O.default_params(w.c_cfl, cascade=3))
    dt = P.initial_dt()
    s, _, _, info = P.step(dt)
    dt = info.dt_next
    s1, vs1, mk, info = P.step(dt, state=P.state)
    assert (mk == 1).sum() > 0 and (mk == 2).sum() > 0 and info.mood_iters >= 3
    s2, vs2, mk2, info2 = P.step(dt, state=P.state, mask=mk, replay=True)
    for a, b in zip((s1.x, s1.vhat, s1.tau, s1.v, s1.e, s1.B), (s2.x, s2.vhat, s2.tau, s2.v, s2.e, s2.B)):
        assert np.array_equal(a, b)
    # the two-level cascade on the same state never uses the limited level
    P2 = O.Problem(w, O.default_params(w.c_cfl, cascade=2))
    _, _, mk2l, _ = P2.step(dt, state=P.state)
    assert set(np.unique(mk2l)) <= {0, 2} and (mk2l == 2).sum() > 0
