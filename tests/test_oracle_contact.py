"""Pins of the oracle's evolving contact boundary condition (Section 3.8,
"Boundary condition treatments"; reading R30): an elastic block falls onto
a rigid slip plane, is held by it, rebounds and detaches.

Fixed by kinematics and mechanics, not by the contact stepper's own formulas: the
step that reaches the plane is cut to the exact impact time gap / U of the
free flight; every node of the flat bottom face lands at once, on the
plane; a slip wall does no work and exerts no tangential force, so total
energy and tangential momentum are conserved through impact and rebound;
nodes in contact do not move normal to the plane and no node passes it;
after the last node detaches the block flies freely (constant momentum);
the whole run is invariant under a rotation of the problem.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import workloads as W

GAP, U = 0.01, 5.0


def _block(v=(0.0, 0.0, -U), Q=None, n=3, detect=True):
    w = W.rotating_cube_3d(n=n, seed=1, omega=0.0)
    w.x = w.x.copy()
    w.x[:, 2] += GAP
    bottom = np.nonzero(np.abs(w.x[:, 2] - GAP) < 1e-12)[0]
    w.v_cell = np.tile(np.asarray(v, float), (w.n_cells, 1))
    w.v_node = np.tile(np.asarray(v, float), (w.n_nodes, 1))
    normal = np.array([0.0, 0.0, 1.0])
    if Q is not None:
        w.x = w.x @ Q.T
        w.v_cell = w.v_cell @ Q.T
        w.v_node = w.v_node @ Q.T
        normal = Q @ normal
    P = O.Problem(w, O.default_params(w.c_cfl, detect=detect))
    return w, P, O.Contact(P, bottom, [0.0, 0.0, 0.0], normal), bottom


def _run(P, K, steps, on_step=None):
    """on_step(k, state, vstar, report, held): held = the nodes in contact
    during the step."""
    dt = P.initial_dt()
    reps = []
    for k in range(steps):
        held = K.contact.copy()
        s, vs, mk, info, rep = K.step(dt)
        reps.append(rep)
        if on_step:
            on_step(k, s, vs, rep, held & K.contact)
        dt = rep["dt_next"]
    return reps


def test_impact_step_is_cut_to_the_exact_impact_time():
    w, P, K, bottom = _block()
    hits = []

    def on(k, s, vs, rep, held):
        if rep["clipped"]:
            hits.append((k, P.t, K.contact.copy(), s.x[bottom, 2].copy()))

    _run(P, K, 8, on)
    assert len(hits) == 1
    k, t, contact, z = hits[0]
    assert t == pytest.approx(GAP / U, rel=1e-12)
    assert contact.all()                          # the flat face lands at once
    assert np.abs(z).max() <= 1e-15


def test_oblique_impact_conserves_energy_and_tangential_momentum():
    w, P, K, bottom = _block(v=(2.0, -1.0, -U))
    d0 = P.diagnostics()
    m = P.m.sum()
    worst = {"below": 0.0, "vn": 0.0}

    def on(k, s, vs, rep, held):
        worst["below"] = min(worst["below"], s.x[bottom, 2].min())
        if held.any():
            worst["vn"] = max(worst["vn"], np.abs(vs[bottom[held], 2]).max())

    reps = _run(P, K, 160, on)
    d1 = P.diagnostics()
    assert any(r["clipped"] for r in reps) and K.contact.sum() == 0
    assert d1["energy"] == pytest.approx(d0["energy"], rel=1e-12)
    assert d1["mom"][0] == pytest.approx(d0["mom"][0], rel=1e-12)
    assert d1["mom"][1] == pytest.approx(d0["mom"][1], rel=1e-12)
    assert d0["mom"][2] == pytest.approx(-U * m, rel=1e-12)
    assert d1["mom"][2] > 0.3 * U * m               # it rebounds
    assert worst["below"] >= -1e-15 and worst["vn"] <= 1e-15 * U


def test_free_flight_after_detachment():
    w, P, K, bottom = _block()
    moms = []

    def on(k, s, vs, rep, held):
        if K.contact.sum() == 0 and k > 20:
            moms.append(P.diagnostics()["mom"][2])

    _run(P, K, 170, on)
    assert len(moms) > 10
    assert np.ptp(moms) <= 1e-12 * abs(moms[0])


def test_rotated_problem_gives_the_rotated_run():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    w, P, K, bottom = _block(v=(1.0, 0.5, -U), detect=False)
    wr, Pr, Kr, _ = _block(v=(1.0, 0.5, -U), Q=Q, detect=False)
    ra = _run(P, K, 40)
    rb = _run(Pr, Kr, 40)
    assert [r["trials"] for r in ra] == [r["trials"] for r in rb]
    assert np.array_equal(K.contact, Kr.contact) and K.contact.any()
    for a, b in zip(ra, rb):
        assert a["dt"] == pytest.approx(b["dt"], rel=1e-11)
    assert np.allclose(Pr.state.x, P.state.x @ Q.T, rtol=0, atol=1e-11)
    assert np.allclose(Pr.state.v, P.state.v @ Q.T, rtol=0, atol=1e-10 * U)
