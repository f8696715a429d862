"""State snapshots (hl_state_save / hl_state_restore): a restored state
steps on bitwise as the original did; a snapshot of another mesh or a
truncated one is refused and leaves the held state as it was."""
import ctypes as C

import numpy as np
import pytest

from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

from .parity_util import FIELDS

pytestmark = pytest.mark.gpu


def _run(ctx, n):
    out = []
    for _ in range(n):
        out.append(ctx.step(0.0))
    return out, ctx.state(), ctx.query("order")


@pytest.mark.parametrize("graph", [False, True])
def test_restore_repeats_the_steps_bitwise(graph):
    w = W.impact_bar_3d(nx=24, ny=6, graded=False)
    ctx = H.from_workload(w)
    ctx.use_graph(graph, 4)
    ctx.compute_dt()
    for _ in range(3):
        ctx.step(0.0)
    blob = ctx.save_state()
    i1, s1, m1 = _run(ctx, 6)
    # change the parameters and the state, then restore
    ctx.set_params(H.default_params(3, c_cfl=0.1, cascade=3))
    ctx.step(0.0)
    ctx.restore_state(blob)
    i2, s2, m2 = _run(ctx, 6)
    for a, b in zip(i1, i2):
        for k in ("dt_used", "dt_next", "mood_iters", "n_p0", "n_recomputed", "energy"):
            assert a[k] == b[k], k
    for f in FIELDS:
        assert np.array_equal(s1[f], s2[f]), f
    assert np.array_equal(m1, m2)


def test_snapshot_of_another_mesh_is_refused():
    w = W.impact_bar_3d(nx=8, ny=3, graded=False)
    a = H.from_workload(w)
    # the same mesh held in the caller's numbering: other connectivity inside
    b = H.Context(0)
    b.set_numbering(H.NUMBERING_KEEP)
    b.upload_mesh(w.dim, w.x, w.cells, w.nwall, w.normals)
    b.init_state(w.rho0, w.mu, w.lam, w.v_cell, w.v_node, H.default_params(3, c_cfl=w.c_cfl))
    c = H.from_workload(W.rotating_cube_3d(n=4))
    blob = a.save_state()
    before = b.state()
    with pytest.raises(H.HyperLagError):
        b.restore_state(blob)
    with pytest.raises(H.HyperLagError):
        c.restore_state(blob)
    with pytest.raises(H.HyperLagError):
        a.restore_state(blob[:-1])
    after = b.state()
    for f in FIELDS:
        assert np.array_equal(before[f], after[f]), f
    # the same mesh in another context: accepted
    a.step(0.0)
    d = H.from_workload(w)
    d.restore_state(a.save_state())
    assert np.array_equal(d.query("x"), a.query("x"))
    assert np.array_equal(d.query("tau"), a.query("tau"))


def test_size_query_and_small_buffer():
    ctx = H.from_workload(W.plane_wave_2d(n=6))
    L = H.load()
    n = C.c_int64()
    assert L.hl_state_save(ctx._h, None, C.byref(n)) == 0 and n.value > 0
    small = C.c_int64(n.value - 1)
    buf = C.create_string_buffer(n.value)
    assert L.hl_state_save(ctx._h, C.cast(buf, C.c_void_p), C.byref(small)) == H.HL_E_INVALID
    assert small.value == n.value
