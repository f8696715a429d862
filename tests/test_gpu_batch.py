"""Batched many-mesh step: one context holds several independent meshes
of uneven size and material; every stage is one launch over all of them
and dt is reduced per mesh.  Each mesh's result must equal, bitwise, the
same mesh stepped alone (and hence the oracle, through the single-mesh
parity tests); one small batch is also checked against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

from .parity_util import FIELDS, err, fmt

pytestmark = pytest.mark.gpu


def _family(dim):
    if dim == 3:
        ws = [W.rotating_cube_3d(n=3, seed=1), W.impact_bar_3d(nx=10, ny=3, graded=False, seed=2),
              W.rotating_cube_3d(n=5, seed=3), W.rotating_cube_3d(n=1, seed=4)]
        ws[2].mu = ws[2].mu * 1.7
        ws[3].v_cell = ws[3].v_cell + 0.3
    else:
        ws = [W.plane_wave_2d(n=6, amp=0.02, seed=5), W.plane_wave_2d(n=17, seed=6),
              W.plane_wave_2d(n=3, amp=0.05, seed=7)]
        ws[1].rho0 = ws[1].rho0 * 2.0
    return ws


def _split(ctx, ws):
    st = ctx.state()
    no, co = ctx.node_offsets, ctx.cell_offsets
    out = []
    for m in range(len(ws)):
        d = {}
        for f in ("x", "vhat"):
            d[f] = st[f][no[m]:no[m + 1]]
        for f in ("tau", "v", "e", "B"):
            d[f] = st[f][co[m]:co[m + 1]]
        out.append(d)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_equals_single_meshes(dim):
    ws = _family(dim)
    print(f"[batch] dim {dim}: sizes {[w.n_cells for w in ws]}", flush=True)
    bctx = H.from_workloads(ws)
    dts_b = bctx.compute_dt()
    singles = [H.from_workload(w) for w in ws]
    for s in singles:
        s.compute_dt()
    steps = 12
    for _ in range(steps):
        bctx.step_batch(None)
        for s in singles:
            s.step(0.0)
    parts = _split(bctx, ws)
    dtb = bctx.next_dt()
    for m, s in enumerate(singles):
        st = s.state()
        for f in FIELDS:
            assert np.array_equal(parts[m][f], st[f]), (m, f)
        assert dtb[m] == s.next_dt()[0]
    assert len(set(np.round(dtb, 15))) > 1, "meshes should take different dt"


def test_batch_explicit_dt_and_oracle():
    ws = _family(3)[:2]
    bctx = H.from_workloads(ws)
    dts = np.array([O.Problem(w).initial_dt() for w in ws]) * 0.5
    bctx.step_batch(dts)
    parts = _split(bctx, ws)
    for m, w in enumerate(ws):
        prob = O.Problem(w)
        s1, _, _, _ = prob.step(dts[m])
        e = {f: err(parts[m][f], getattr(s1, f)) for f in FIELDS}
        assert max(e.values()) <= 1e-12, fmt(e)


def test_batch_rejects_bad_offsets():
    ws = _family(2)[:2]
    ctx = H.Context(0)
    x = np.concatenate([w.x for w in ws])
    cells = np.concatenate([w.cells for w in ws])
    with pytest.raises(H.HyperLagError):
        # second mesh's cells refer past its own nodes
        ctx.upload_mesh_batch(2, [0, ws[0].n_nodes, ws[0].n_nodes + 3],
                              [0, ws[0].n_cells, ws[0].n_cells + ws[1].n_cells], x[:ws[0].n_nodes + 3],
                              cells)
