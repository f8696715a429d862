"""Stiffened-gas equation of state (hl_params.eos = 1; eq.
EOS_stiffened_gas with the shear family; reading R31) through the C-ABI
against the oracle: one-step parity with a = -1 and a = 0 in 3D and 2D, a
100-step impact run with identical cascades, the stress query, the energy
diagnostics and the parameter checks."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

from .parity_util import compare_states, fmt, max_err

pytestmark = pytest.mark.gpu

ONE_STEP = 1e-12
HUNDRED = 1e-9
GAM, PINF = 2.2, 1e6


def _jelly_bar():
    """The droplet test's material (rho0 = 1020, mu = 85, gamma = 2.2,
    p_inf = 1e6) as a bar hitting the slip wall x = 0 at 3 m/s."""
    w = W.impact_bar_3d(nx=16, ny=4, graded=True, seed=11, v0=-3.0)
    w.rho0 = np.full(w.n_cells, 1020.0)
    w.mu = np.full(w.n_cells, 85.0)
    return w, PINF


def _gas_cube():
    w = W.rotating_cube_3d(n=5, seed=2, omega=20.0)
    w.rho0 = np.full(w.n_cells, 1020.0)
    w.mu = np.full(w.n_cells, 2e4)
    return w, PINF


def _gas_square():
    w = W.plane_wave_2d(n=16, amp=0.05)
    return w, 1.0


CASES = {"jelly_bar": _jelly_bar, "gas_cube": _gas_cube, "gas_square": _gas_square}


def _pair(w, pinf, a=-1.0):
    gp = H.default_params(w.dim, c_cfl=w.c_cfl, shear_a=a, eos=1, sg_gamma=GAM, sg_pinf=pinf)
    op = O.default_params(w.c_cfl, shear_a=a, eos=1, sg_gamma=GAM, sg_pinf=pinf)
    return H.from_workload(w, params=gp), O.Problem(w, op)


@pytest.mark.parametrize("a", [-1.0, 0.0])
@pytest.mark.parametrize("case", list(CASES))
def test_one_step_parity_stiffened_gas(case, a):
    w, pinf = CASES[case]()
    ctx, prob = _pair(w, pinf, a)
    assert np.allclose(ctx.state()["e"], prob.state.e, rtol=1e-15, atol=0)
    dt = prob.initial_dt()
    assert ctx.compute_dt() == pytest.approx(dt, rel=1e-13)
    ctx.step(dt)
    _, _, mk0, oi0 = prob.step(dt)
    assert np.array_equal(ctx.query("order"), mk0)
    dt = oi0.dt_next
    info = ctx.step(dt)
    s1, vs, mk, oi = prob.step(dt)
    e = compare_states(ctx, s1, vs)
    print(f"[gas a={a}] {case}: {fmt(e)} p0 {info['n_p0']}/{oi.n_p0}", flush=True)
    assert np.array_equal(ctx.query("order"), mk)
    assert max_err(e) <= ONE_STEP, fmt(e)
    assert math.isclose(info["energy"], oi.energy, rel_tol=1e-12)
    assert info["dt_next"] == pytest.approx(oi.dt_next, rel=1e-12)


def test_jelly_bar_hundred_steps():
    w, pinf = _jelly_bar()
    ctx, prob = _pair(w, pinf)
    ctx.compute_dt()
    dt = prob.initial_dt()
    flips, p0 = 0, 0
    for _ in range(100):
        ctx.step(0.0)
        _, _, mk, oi = prob.step(dt)
        flips += int(not np.array_equal(ctx.query("order"), mk))
        p0 += oi.n_p0
        dt = oi.dt_next
    e = compare_states(ctx, prob.state)
    print(f"[gas] jelly bar 100 steps: {fmt(e)} mask-differing steps {flips}, p0 cell-steps {p0}", flush=True)
    assert flips == 0
    assert max_err(e) <= HUNDRED, fmt(e)


@pytest.mark.parametrize("a", [-1.0, 0.0])
def test_stress_query_and_stored_energy(a):
    w, pinf = _gas_cube()
    ctx, prob = _pair(w, pinf, a)
    for _ in range(3):
        ctx.step(0.0)
    st = ctx.state()
    T = ctx.query("T")
    for c in (0, 17, w.n_cells - 1):
        B = np.array([[st["B"][c, 0], st["B"][c, 3], st["B"][c, 4]],
                      [st["B"][c, 3], st["B"][c, 1], st["B"][c, 5]],
                      [st["B"][c, 4], st["B"][c, 5], st["B"][c, 2]]])
        eps = st["e"][c] - 0.5 * np.sum(st["v"][c] ** 2)
        To, p, _, _ = O.point_stress_sg(prob.rho0[c], prob.mu[c], st["tau"][c], B, eps, a, GAM, pinf)
        ref = np.array([To[0, 0], To[1, 1], To[2, 2], To[0, 1], To[0, 2], To[1, 2]])
        # the pressure is a difference of terms of size gamma p_inf
        assert np.allclose(T[c], ref, rtol=0, atol=1e-13 * GAM * pinf)
    info = ctx.step(0.0)
    od = prob.diagnostics(O.State(*(ctx.state()[f] for f in ("x", "vhat", "tau", "v", "e", "B"))))
    assert info["elastic"] == pytest.approx(od["elastic"], rel=1e-11, abs=1e-14 * info["energy"])


def test_stiffened_gas_parameter_checks():
    w, pinf = _gas_cube()
    ctx = H.from_workload(w)
    for kw in (dict(eos=1, sg_gamma=1.0), dict(eos=1, sg_pinf=-1.0), dict(eos=1, cascade=3), dict(eos=2)):
        with pytest.raises(H.HyperLagError):
            ctx.set_params(H.default_params(3, **kw))
    ctx.set_params(H.default_params(3, eos=1))
    with pytest.raises(H.HyperLagError):
        ctx.forward_record(2, 1)
