"""Pins of the oracle's shear energy family (Section 2.2.4, eq.
familiy_energies, with the stress of eqs. T_psi / cst):

    Psi_s = mu/(4 rho0) [-2a (I1b - 3) + (1+a)/3 (I2b^2 - 9)],
    T = -p I + 2 rho [dPsi_s/dI1b dev(Bbar) - dPsi_s/dI2b dev(Bbar^-1)].

The stress is checked against finite differences of the oracle's own
energy function (a separately written formula): on states with det Bbar = 1
the deviatoric stress equals dev(2 rho (dPsi/dB) B), the general
hyperelastic relation.  Further pins: frame indifference, the family's
small-strain shear modulus mu for every a, the directional derivative
against finite differences of the stress, continuity at a = -1 (the
neo-Hookean member) and conservation with the GCL in a full step.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import workloads as W

from .test_oracle_pins import _gcl_defect

RHO0, MU, K = 1100.0, 8.2e5, 3.9e6 + 2 * 8.2e5 / 3
AS = [-0.5, 0.0, 0.25, 0.5]


def _spd_unimodular(rng, amp):
    A = np.eye(3) + amp * rng.uniform(-1, 1, (3, 3))
    U = A @ A.T
    return U / np.linalg.det(U) ** (1.0 / 3.0)


def _dev(T):
    return T - np.trace(T) / 3.0 * np.eye(3)


@pytest.mark.parametrize("a", AS)
def test_stress_is_the_energy_derivative(a):
    rng = np.random.default_rng(11)
    for _ in range(10):
        tau = rng.uniform(0.8, 1.2) / RHO0
        J = RHO0 * tau
        B = J ** (2.0 / 3.0) * _spd_unimodular(rng, 0.3)      # det Bbar = 1
        T, _, _, _ = O.point_stress(RHO0, MU, K, tau, B, a)
        psi = lambda Bx: O.point_stress(RHO0, MU, K, tau, Bx, a)[3]
        G = np.zeros((3, 3))
        for i in range(3):
            for j in range(i, 3):
                h = 1e-6 * np.abs(B).max()
                E = np.zeros((3, 3))
                E[i, j] = E[j, i] = 1.0
                d = (psi(B + h * E) - psi(B - h * E)) / (2 * h)
                G[i, j] = G[j, i] = d if i == j else 0.5 * d
        Tfd = 2.0 / tau * G @ B
        scale = np.abs(_dev(T)).max()
        assert np.allclose(_dev(T), _dev(Tfd), rtol=0, atol=2e-7 * scale)


@pytest.mark.parametrize("a", AS)
def test_frame_indifference(a):
    rng = np.random.default_rng(12)
    for _ in range(5):
        tau = rng.uniform(0.8, 1.2) / RHO0
        B = _spd_unimodular(rng, 0.4) * rng.uniform(0.9, 1.1)
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        T, _, _, _ = O.point_stress(RHO0, MU, K, tau, B, a)
        TQ, _, _, _ = O.point_stress(RHO0, MU, K, tau, Q @ B @ Q.T, a)
        assert np.allclose(TQ, Q @ T @ Q.T, rtol=0, atol=1e-12 * np.abs(T).max())


@pytest.mark.parametrize("a", AS + [-1.0])
def test_small_strain_shear_modulus_is_mu(a):
    """Simple shear F = I + g e1 (x) e2 at J = 1: T12 = mu g + O(g^2) for every
    member of the family."""
    for g in (1e-4, 1e-5):
        B = np.array([[1.0 + g * g, g, 0.0], [g, 1.0, 0.0], [0.0, 0.0, 1.0]])
        T, _, _, _ = O.point_stress(RHO0, MU, K, 1.0 / RHO0, B, a)
        assert T[0, 1] / g == pytest.approx(MU, rel=5 * g)


@pytest.mark.parametrize("a", AS)
def test_stress_direction_is_the_derivative(a):
    rng = np.random.default_rng(13)
    for _ in range(5):
        tau = rng.uniform(0.8, 1.2) / RHO0
        B = _spd_unimodular(rng, 0.3) * rng.uniform(0.9, 1.1)
        dB = rng.standard_normal((3, 3))
        dB = 0.5 * (dB + dB.T)
        dtau = rng.standard_normal() * tau
        dT = O.point_stress_direction(RHO0, MU, K, tau, B, dtau, dB, a)
        h = 1e-6
        Tp = O.point_stress(RHO0, MU, K, tau + h * dtau, B + h * dB, a)[0]
        Tm = O.point_stress(RHO0, MU, K, tau - h * dtau, B - h * dB, a)[0]
        fd = (Tp - Tm) / (2 * h)
        assert np.allclose(dT, fd, rtol=0, atol=1e-6 * np.abs(fd).max())


def test_neo_hookean_is_the_family_member_a_minus_one():
    rng = np.random.default_rng(14)
    tau = 1.05 / RHO0
    B = _spd_unimodular(rng, 0.3) * 1.02
    T1, _, _, psi1 = O.point_stress(RHO0, MU, K, tau, B, -1.0)
    T2, _, _, psi2 = O.point_stress(RHO0, MU, K, tau, B, -1.0 + 1e-9)
    assert np.allclose(T1, T2, rtol=0, atol=1e-7 * np.abs(T1).max())
    assert psi2 == pytest.approx(psi1, rel=1e-7)


@pytest.mark.parametrize("a", [0.0, 0.5])
def test_step_with_the_family_conserves_and_keeps_the_gcl(a):
    w = W.impact_bar_3d(nx=12, ny=3, graded=False)
    P = O.Problem(w, O.default_params(w.c_cfl, shear_a=a))
    d0 = P.diagnostics()
    dt = P.initial_dt()
    for _ in range(4):
        x0 = P.state.x.copy()
        s1, vstar, mk, info = P.step(dt)
        assert _gcl_defect(w, x0, s1.x, vstar, dt, None) < 1e-12
        dt = info.dt_next
    d1 = P.diagnostics()
    assert d1["mass"] == d0["mass"]
    assert d1["energy"] == pytest.approx(d0["energy"], rel=1e-13)
    assert np.all(np.isfinite(P.state.B))
