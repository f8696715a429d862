"""Pins of the oracle's stiffened-gas equation of state (eq.
EOS_stiffened_gas with the shear family; reading R31):

    eps_v = eps - Psi_s = (p + gamma p_inf) / ((gamma - 1) rho).

Fixed by thermodynamics and mechanics, not by the oracle's own formulas:
the pressure satisfies the paper's printed relation; the sound speed is
the isentropic one, -tau^2 dp/dtau along d eps = -p d tau (finite
differences); the equation of state only changes the isotropic part of
the stress; the directional derivative used by the predictor matches
finite differences of the stress in (tau, B, eps); the predicted corner
state of a uniform affine flow is the exact state at t + dt/2 (the ODEs
d tau/dt = tau tr G, d eps/dt = tau T : G, dB/dt = G B + B G^T integrated
by RK4 in the test); a body at rest stays at rest; full steps conserve
mass and total energy and keep the GCL; with gamma p_inf equal to the
solid's bulk modulus, small-amplitude waves match the neo-Hookean solid.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import workloads as W

from .test_oracle_pins import _gcl_defect

RHO0, MU, GAM, PINF = 1020.0, 85.0, 2.2, 1e6


def _unimodular(rng, amp):
    A = np.eye(3) + amp * rng.uniform(-1, 1, (3, 3))
    U = A @ A.T
    return U / np.linalg.det(U) ** (1.0 / 3.0)


def _dev(T):
    return T - np.trace(T) / 3.0 * np.eye(3)


@pytest.mark.parametrize("a", [-1.0, 0.0])
def test_pressure_satisfies_the_printed_relation(a):
    rng = np.random.default_rng(1)
    for _ in range(10):
        tau = rng.uniform(0.9, 1.1) / RHO0
        J = RHO0 * tau
        B = J ** (2.0 / 3.0) * _unimodular(rng, 0.2)
        eps = rng.uniform(1.0, 2.0) * GAM * PINF * tau / (GAM - 1.0)
        T, p, _, psi = O.point_stress_sg(RHO0, 2e4, tau, B, eps, a, GAM, PINF)
        eps_v = (p + GAM * PINF) / ((GAM - 1.0) / tau)       # (p + g p_inf) / ((g - 1) rho)
        assert eps_v == pytest.approx(eps - psi, rel=1e-13)
        assert np.trace(T) / 3.0 == pytest.approx(-p, rel=1e-12, abs=1e-9 * PINF)


def test_sound_speed_is_the_isentropic_one():
    rng = np.random.default_rng(2)
    for _ in range(5):
        tau = rng.uniform(0.9, 1.1) / RHO0
        B = (RHO0 * tau) ** (2.0 / 3.0) * np.eye(3)          # no shear energy
        eps = rng.uniform(1.0, 1.5) * GAM * PINF * tau / (GAM - 1.0)
        _, p, a, _ = O.point_stress_sg(RHO0, 0.0, tau, B, eps, -1.0, GAM, PINF)
        h = 1e-5 * tau
        pp = O.point_stress_sg(RHO0, 0.0, tau + h, B, eps - p * h, -1.0, GAM, PINF)[1]
        pm = O.point_stress_sg(RHO0, 0.0, tau - h, B, eps + p * h, -1.0, GAM, PINF)[1]
        c2 = -tau * tau * (pp - pm) / (2.0 * h)
        assert a * a == pytest.approx(c2, rel=1e-7)
        # the shear adds 4 mu / 3 to the longitudinal modulus
        _, _, a_mu, _ = O.point_stress_sg(RHO0, MU, tau, B, eps, -1.0, GAM, PINF)
        assert a_mu * a_mu - a * a == pytest.approx(tau * 4.0 * MU / 3.0, rel=1e-9)


@pytest.mark.parametrize("a", [-1.0, 0.0, 0.5])
def test_equation_of_state_changes_only_the_isotropic_part(a):
    rng = np.random.default_rng(3)
    for _ in range(5):
        tau = rng.uniform(0.9, 1.1) / RHO0
        B = _unimodular(rng, 0.3) * rng.uniform(0.95, 1.05)
        eps = 2.0 * GAM * PINF * tau / (GAM - 1.0)
        Tsg = O.point_stress_sg(RHO0, 3e3, tau, B, eps, a, GAM, PINF)[0]
        Tnh = O.point_stress(RHO0, 3e3, 4e6, tau, B, a)[0]
        assert np.allclose(_dev(Tsg), _dev(Tnh), rtol=0, atol=1e-12 * np.abs(_dev(Tnh)).max())


@pytest.mark.parametrize("a", [-1.0, 0.0])
def test_stress_direction_is_the_derivative(a):
    rng = np.random.default_rng(4)
    for _ in range(5):
        tau = rng.uniform(0.9, 1.1) / RHO0
        B = _unimodular(rng, 0.3) * rng.uniform(0.95, 1.05)
        eps = 1.5 * GAM * PINF * tau / (GAM - 1.0)
        dB = rng.standard_normal((3, 3))
        dB = 0.5 * (dB + dB.T)
        dtau, deps = rng.standard_normal() * tau, rng.standard_normal() * eps
        dT = O.point_stress_direction_sg(RHO0, 5e4, tau, B, eps, dtau, dB, deps, a, GAM, PINF)
        h = 1e-6
        Tp = O.point_stress_sg(RHO0, 5e4, tau + h * dtau, B + h * dB, eps + h * deps, a, GAM, PINF)[0]
        Tm = O.point_stress_sg(RHO0, 5e4, tau - h * dtau, B - h * dB, eps - h * deps, a, GAM, PINF)[0]
        fd = (Tp - Tm) / (2 * h)
        assert np.allclose(dT, fd, rtol=0, atol=1e-6 * np.abs(fd).max())


def _gas_cube(n=3, omega=0.0, **kw):
    w = W.rotating_cube_3d(n=n, seed=4, omega=omega)
    w.rho0 = np.full(w.n_cells, RHO0)
    w.mu = np.full(w.n_cells, MU)
    prm = O.default_params(w.c_cfl, eos=1, sg_gamma=GAM, sg_pinf=PINF, **kw)
    return w, O.Problem(w, prm)


def test_predicted_corner_state_of_an_affine_flow():
    """Uniform state, v = G x: the corner state is the state at dt / 2
    advanced by one Euler step of the flow's ODEs, so its error against the
    exact state (RK4 in the test) falls as dt^2."""
    w, P = _gas_cube(n=2)
    G = np.array([[0.3, 0.1, -0.05], [0.02, -0.2, 0.1], [0.05, 0.04, 0.15]]) * 50.0
    s = P.state.copy()
    xc = s.x[w.cells].mean(axis=1)
    s.v = xc @ G.T
    # uniform eps with p = gamma p_inf / 2, so the flow does work from t = 0
    s.e = 1.5 * GAM * PINF * s.tau / (GAM - 1.0) + 0.5 * np.sum(s.v ** 2, axis=1)
    tau0, eps0 = s.tau[0], s.e[0] - 0.5 * np.sum(s.v[0] ** 2)

    def rhs(y):
        tau, eps, B = y[0], y[1], y[2:].reshape(3, 3)
        T = O.point_stress_sg(RHO0, MU, tau, B, eps, -1.0, GAM, PINF)[0]
        return np.concatenate([[tau * np.trace(G), tau * np.sum(T * G)], (G @ B + B @ G.T).ravel()])

    errs = []
    for dt in (8e-4, 4e-4, 2e-4):
        y = np.concatenate([[tau0, eps0], np.eye(3).ravel()])
        n = 100
        hh = 0.5 * dt / n
        for _ in range(n):
            k1 = rhs(y)
            k2 = rhs(y + 0.5 * hh * k1)
            k3 = rhs(y + 0.5 * hh * k2)
            k4 = rhs(y + hh * k3)
            y = y + hh / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        T_exact = O.point_stress_sg(RHO0, MU, y[0], y[2:].reshape(3, 3), y[1], -1.0, GAM, PINF)[0]
        ts, es, Ts, zs = P.predict_eos(dt, state=s)
        assert np.allclose(es, es[0, 0], rtol=1e-13) and np.allclose(ts, ts[0, 0], rtol=1e-13)
        errs.append((abs(es[0, 0] - y[1]) / abs(y[1] - eps0), np.abs(Ts[0, 0] - T_exact).max(),
                     abs(ts[0, 0] - y[0]) / abs(y[0] - tau0)))
    for k in range(2):
        for j in range(3):
            ratio = errs[k + 1][j] / errs[k][j]
            assert 0.2 < ratio < 0.3 if j == 1 else 0.4 < ratio < 0.6, (k, j, errs)


def test_body_at_rest_stays_at_rest():
    w, P = _gas_cube(n=3)
    w.v_cell = w.v_cell * 0.0
    w.v_node = w.v_node * 0.0
    P = O.Problem(w, P.params)
    dt = P.initial_dt()
    e0 = P.state.e.copy()
    s1, vs, mk, info = P.step(dt)
    scale = np.sqrt(GAM * PINF / RHO0)
    assert np.abs(vs).max() <= 1e-12 * scale
    assert np.allclose(s1.e, e0, rtol=1e-14, atol=0)
    assert info.n_p0 == 0


def test_steps_conserve_and_keep_the_gcl():
    w, P = _gas_cube(n=3, omega=30.0)
    d0 = P.diagnostics()
    dt = P.initial_dt()
    for _ in range(6):
        x0 = P.state.x.copy()
        s1, vstar, mk, info = P.step(dt)
        assert _gcl_defect(w, x0, s1.x, vstar, dt, None) < 1e-12
        dt = info.dt_next
    d1 = P.diagnostics()
    assert d1["mass"] == d0["mass"]
    assert d1["energy"] == pytest.approx(d0["energy"], rel=1e-13)
    assert np.all(np.isfinite(P.state.e))


def test_small_waves_match_the_solid_with_the_same_bulk_modulus():
    """gamma p_inf = K: the stiffened gas at p = 0 linearises to the solid's
    acoustics, so a small plane wave evolves alike in both."""
    w = W.plane_wave_2d(n=16, amp=1e-6, seed=1)
    K = w.lam[0] + 2.0 * w.mu[0] / 3.0
    Pn = O.Problem(w, O.default_params(w.c_cfl, detect=False))
    Ps = O.Problem(w, O.default_params(w.c_cfl, detect=False, eos=1, sg_gamma=GAM, sg_pinf=K / GAM))
    dt = Pn.initial_dt()
    assert Ps.initial_dt() == pytest.approx(dt, rel=1e-12)
    for _ in range(40):
        Pn.step(dt)
        Ps.step(dt)
    vn, vs = Pn.state.v, Ps.state.v
    assert np.abs(vn).max() > 1e-8
    assert np.abs(vs - vn).max() <= 1e-4 * np.abs(vn).max()
