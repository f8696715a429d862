"""Conforming red refinement on the GPU (hl_mesh_refine; Section 3.9)
against the oracle's refinement: node positions, cells, wall counts and
normals bit for bit, one and two levels, 3D and 2D; then the step on a
refined mesh against the oracle; the argument checks."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

from .parity_util import compare_states, fmt, max_err

pytestmark = pytest.mark.gpu

CASES = {
    "bar_24x6": lambda: W.impact_bar_3d(nx=24, ny=6, graded=False, seed=5),
    "cube_n3": lambda: W.rotating_cube_3d(n=3, seed=3),
    "square_n10": lambda: W.plane_wave_2d(n=10, seed=2),
}


def _refined_workload(w, levels):
    x, cells, nwall, normals = O.refine(w.dim, w.x, w.cells, w.nwall, w.normals, levels)
    k = (8 if w.dim == 3 else 4) ** levels
    rep = lambda a: np.repeat(a, k, axis=0)
    vn = np.tile(w.v_node[:1], (len(x), 1))      # uniform node velocity
    return W.Workload(w.name + f"_r{levels}", w.dim, x, cells, nwall, normals, rep(w.rho0), rep(w.mu),
                      rep(w.lam), rep(w.v_cell), vn, w.c_cfl, w.steps)


@pytest.mark.parametrize("case,levels", [("bar_24x6", 1), ("cube_n3", 1), ("cube_n3", 2), ("square_n10", 1),
                                          ("square_n10", 2)])
def test_refinement_matches_the_oracle(case, levels):
    w = CASES[case]()
    ctx = H.Context()
    ctx.upload_mesh(w.dim, w.x, w.cells, w.nwall, w.normals)
    ctx.refine(levels)
    g = ctx.mesh()
    x, cells, nwall, normals = O.refine(w.dim, w.x, w.cells, w.nwall, w.normals, levels)
    print(f"[refine] {case} x{levels}: {w.n_cells} -> {ctx.n_cells} cells, {ctx.n_nodes} nodes", flush=True)
    assert np.array_equal(g["x"], x)
    assert np.array_equal(g["cells"], cells)
    assert np.array_equal(g["nwall"], nwall)
    assert np.array_equal(g["normals"], normals)


def test_step_on_a_refined_bar():
    """The impact bar (uniform velocity into its x = 0 wall) refined once:
    the refined walls hold and the step matches the oracle's."""
    w = W.impact_bar_3d(nx=12, ny=3, graded=False, seed=7)
    wr = _refined_workload(w, 1)
    ctx = H.Context()
    ctx.upload_mesh(w.dim, w.x, w.cells, w.nwall, w.normals)
    ctx.refine(1)
    H.init_from_workloads(ctx, [wr])
    prob = O.Problem(wr)
    dt = prob.initial_dt()
    ctx.step(dt)
    s1, vs, mk, oi = prob.step(dt)
    e = compare_states(ctx, s1, vs)
    assert np.array_equal(ctx.query("order"), mk)
    assert max_err(e) <= 1e-12, fmt(e)
    dt = oi.dt_next
    for _ in range(30):
        ctx.step(dt)
        _, _, mk, oi = prob.step(dt)
        assert np.array_equal(ctx.query("order"), mk)
        dt = oi.dt_next
    e = compare_states(ctx, prob.state)
    print(f"[refine] bar x1, 31 steps: {fmt(e)}", flush=True)
    assert max_err(e) <= 1e-9, fmt(e)
    wall = wr.nwall > 0
    assert np.abs(ctx.query("vstar")[wall, 0]).max() == 0.0


def test_refinement_checks():
    w = CASES["cube_n3"]()
    ctx = H.from_workload(w)
    with pytest.raises(H.HyperLagError):
        ctx.refine(5)
    ctx.refine(0)
    assert ctx.n_cells == w.n_cells
    ctx.refine(1)
    with pytest.raises(H.HyperLagError):
        ctx.step(1e-6)                 # the state went with the old mesh
    bctx = H.from_workloads([w, w])
    with pytest.raises(H.HyperLagError):
        bctx.refine(1)
