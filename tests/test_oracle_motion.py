"""Pins of the oracle's free-flight motion in uniform static E and B (classical equations
of motion, the paper's UniformFieldClassic; swarm geometry: z along E, B in the xz plane)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import synth

QE, ME, AMU = oracle.constants()


def _model(E, B=0.0, ang=0.0):
    return oracle.OracleModel([synth.maxwell_component(4.0)], E, B, ang)


def _lorentz(E, B, ang):
    Evec = np.array([0.0, 0.0, E])
    Bvec = B * np.array([math.sin(ang), 0.0, math.cos(ang)])

    def f(_t, y):
        v = y[3:]
        acc = (-QE / ME) * (Evec + np.cross(v, Bvec))
        return np.concatenate([v, acc])
    return f


def test_no_magnetic_field_is_uniform_acceleration():
    E = 2.5e5
    m = _model(E)
    rng = np.random.default_rng(0)
    for _ in range(20):
        r0 = rng.normal(size=3) * 1e-3
        v0 = rng.normal(size=3) * 1e6
        T = rng.uniform(0, 5e-12)
        r, v = m.move(r0, v0, T)
        a = np.array([0.0, 0.0, -QE * E / ME])
        np.testing.assert_allclose(v, v0 + a * T, rtol=1e-14, atol=1e-9)
        np.testing.assert_allclose(r, r0 + v0 * T + 0.5 * a * T * T, rtol=1e-14, atol=1e-20)


@pytest.mark.parametrize("E,B,ang", [(2.5e5, 1.0, math.pi / 4), (1e6, 2.0, math.pi / 2),
                                     (0.0, 1.5, 0.3), (5e4, 0.5, 2.5)])
def test_crossed_fields_match_numerical_integration(E, B, ang):
    m = _model(E, B, ang)
    rng = np.random.default_rng(1)
    omega = QE * B / ME
    period = 2 * math.pi / omega
    for _ in range(3):
        r0 = rng.normal(size=3) * 1e-4
        v0 = rng.normal(size=3) * 5e5
        for T in (0.013 * period, 0.7 * period, 3.3 * period, 10.0 * period):
            sol = solve_ivp(_lorentz(E, B, ang), (0, T), np.concatenate([r0, v0]), method="DOP853",
                            rtol=1e-12, atol=1e-22)
            r, v = m.move(r0, v0, T)
            scale_v = np.linalg.norm(v0) + QE * E / ME * T + 1.0
            scale_r = np.linalg.norm(v0) * T + QE * E / ME * T * T + 1e-12
            assert np.max(np.abs(v - sol.y[3:, -1])) < 1e-8 * scale_v
            assert np.max(np.abs(r - sol.y[:3, -1])) < 1e-8 * scale_r


def test_cyclotron_period_and_gyroradius():
    B, ang = 1.0, 0.4
    m = _model(0.0, B, ang)
    omega = QE * B / ME
    bhat = np.array([math.sin(ang), 0.0, math.cos(ang)])
    v0 = np.array([3e5, -2e5, 1e5])
    T = 2 * math.pi / omega
    r, v = m.move(np.zeros(3), v0, T)
    np.testing.assert_allclose(v, v0, rtol=0, atol=1e-9 * np.linalg.norm(v0))
    np.testing.assert_allclose(r, bhat * np.dot(v0, bhat) * T, rtol=0, atol=1e-9 * np.linalg.norm(v0) * T)
    # distance from the guiding centre stays |u0|/omega
    u0 = v0 - bhat * np.dot(v0, bhat)
    rho = np.linalg.norm(u0) / omega
    centre = np.cross(bhat, u0) / omega
    for f in (0.1, 0.37, 0.5, 0.81):
        rr, _ = m.move(np.zeros(3), v0, f * T)
        perp = rr - bhat * np.dot(rr, bhat)
        assert abs(np.linalg.norm(perp - centre) - rho) < 1e-9 * rho


def test_guiding_centre_drift_is_E_cross_B():
    E, B = 2e5, 1.0
    m = _model(E, B, math.pi / 2)    # B along x, perpendicular to E
    omega = QE * B / ME
    T = 2 * math.pi / omega
    r, _ = m.move(np.zeros(3), np.array([0.0, 2e5, -3e5]), 5 * T)   # no velocity along B
    vD = np.cross([0, 0, E], [B, 0, 0]) / B ** 2
    np.testing.assert_allclose(r / (5 * T), vD, rtol=0, atol=1e-9 * np.linalg.norm(vD) + 1e-6)


@pytest.mark.parametrize("B,ang", [(0.0, 0.0), (1.0, math.pi / 4), (2.0, 1.2)])
def test_free_flight_energy_equals_work_of_E(B, ang):
    # eps(T) - eps(0) = -E * (z(T) - z0) in eV (charge -e); B does no work
    E = 3e5
    m = _model(E, B, ang)
    rng = np.random.default_rng(2)
    for _ in range(50):
        v0 = rng.normal(size=3) * 1e6
        T = rng.uniform(0, 2e-11)
        r, v = m.move(np.zeros(3), v0, T)
        e0 = 0.5 * ME * v0 @ v0 / QE
        e1 = 0.5 * ME * v @ v / QE
        assert abs((e1 - e0) - (-E * r[2])) < 1e-9 * max(e0, e1, 1e-3)
