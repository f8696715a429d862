"""Rigid-plane contact (hl_set_contact; Section 3.8, reading R30) through
the C-ABI against the oracle's contact stepper: an elastic block falls onto
the plane, is held, rebounds and detaches (3D, oblique, and a 2D square),
with the same trial sequence, cut steps, contact states and cascade masks
at every step; graph capture; the argument checks."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

from .parity_util import FIELDS, compare_states, fmt, max_err
from .test_oracle_contact import GAP, U, _block

pytestmark = pytest.mark.gpu

MANY = 1e-9


def _square(v=(0.1, -0.5)):
    w = W.plane_wave_2d(n=8, amp=0.0, seed=2)
    w.nwall = np.zeros_like(w.nwall)
    w.normals = np.zeros_like(w.normals)
    w.x = w.x.copy()
    w.x[:, 1] += GAP
    bottom = np.nonzero(np.abs(w.x[:, 1] - GAP) < 1e-12)[0]
    w.v_cell = np.tile(np.asarray(v, float), (w.n_cells, 1))
    w.v_node = np.tile(np.asarray(v, float), (w.n_nodes, 1))
    P = O.Problem(w, O.default_params(w.c_cfl))
    return w, P, O.Contact(P, bottom, [0.0, 0.0], [0.0, 1.0]), bottom


def _gpu(w, bottom, normal):
    ctx = H.from_workload(w)
    ctx.set_contact(bottom.astype(np.int32), np.zeros(w.dim), normal)
    return ctx


def _compare_run(w, P, K, bottom, normal, steps, tag):
    ctx = _gpu(w, bottom, normal)
    dt = P.initial_dt()
    ctx.compute_dt()
    events = 0
    for k in range(steps):
        info = ctx.step(0.0)
        _, _, mk, oi, rep = K.step(dt)
        assert info["trials"] == rep["trials"] and bool(info["clipped"]) == rep["clipped"], (k, info, rep)
        assert info["dt_used"] == pytest.approx(rep["dt"], rel=1e-12), k
        assert info["dt_next"] == pytest.approx(rep["dt_next"], rel=1e-12), k
        assert np.array_equal(ctx.contact_state(), K.contact), k
        assert np.array_equal(ctx.query("order"), mk), k
        events += rep["trials"] > 1
        dt = rep["dt_next"]
    e = compare_states(ctx, P.state)
    print(f"[contact {tag}] {steps} steps, {events} redone: {fmt(e)}", flush=True)
    assert max_err(e) <= MANY, fmt(e)
    return ctx, events


@pytest.mark.parametrize("v", [(0.0, 0.0, -U), (2.0, -1.0, -U)])
def test_block_impact_rebound_parity(v):
    w, P, K, bottom = _block(v=v)
    ctx, events = _compare_run(w, P, K, bottom, [0.0, 0.0, 1.0], 160, f"block v={v}")
    assert events >= 3 and K.contact.sum() == 0 and P.state.v[:, 2].mean() > 0


def test_square_impact_parity_2d():
    w, P, K, bottom = _square()
    ctx, events = _compare_run(w, P, K, bottom, [0.0, 1.0], 120, "square")
    assert events >= 2


def test_contact_with_graph_equals_eager():
    w, P, K, bottom = _block(v=(1.0, 0.0, -U))
    eager = _gpu(w, bottom, [0.0, 0.0, 1.0])
    graph = _gpu(w, bottom, [0.0, 0.0, 1.0])
    graph.use_graph(True, 6)
    for c in (eager, graph):
        c.compute_dt()
    for k in range(60):
        ie, ig = eager.step(0.0), graph.step(0.0)
        assert ie["trials"] == ig["trials"] and ie["dt_used"] == ig["dt_used"], k
        se, sg = eager.state(), graph.state()
        for f in FIELDS:
            assert np.array_equal(se[f], sg[f]), (k, f)
        assert np.array_equal(eager.contact_state(), graph.contact_state()), k


def test_contact_checks_and_release():
    w, P, K, bottom = _block()
    ctx = H.from_workload(w)
    b = bottom.astype(np.int32)
    for args in ((np.array([w.n_nodes], np.int32), [0, 0, 0], [0, 0, 1]),
                 (np.array([b[0], b[0]], np.int32), [0, 0, 0], [0, 0, 1]),
                 (b, [0, 0, 0], [0, 0, 0]),
                 (b, [0, 0, np.nan], [0, 0, 1])):
        with pytest.raises(H.HyperLagError):
            ctx.set_contact(*args)
    ctx.set_contact(b, [0, 0, 0], [0, 0, 1])
    with pytest.raises(H.HyperLagError):
        ctx.forward_record(2, 1)
    ctx.compute_dt()
    for _ in range(8):
        ctx.step(0.0)
    assert ctx.contact_state().all()
    # a new state releases the candidates
    H.init_from_workloads(ctx, [w])
    assert not ctx.contact_state().any()
    # removal restores the own walls: steps equal a context that never had contact
    ctx.set_contact()
    plain = H.from_workload(w)
    dt = plain.compute_dt()
    for _ in range(8):
        ctx.step(dt)
        plain.step(dt)
    a, b2 = ctx.state(), plain.state()
    for f in FIELDS:
        assert np.array_equal(a[f], b2[f]), f
    # a batch context refuses contact
    bctx = H.from_workloads([w, w])
    with pytest.raises(H.HyperLagError):
        bctx.set_contact(b, [0, 0, 0], [0, 0, 1])
