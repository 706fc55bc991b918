"""Pins of the oracle's relativistic mover (section "Theoretical framework" and the
UniformFieldRelativisticChin field of section "Software architecture", uniform static E and
B): the motion against a numerical integration of the relativistic Lorentz force,
hyperbolic motion from rest, the relativistic cyclotron period, the classical limits of both
movers, the work-energy theorem (B does no work), the electron speed at the rest energy, and
whole runs that reduce to the classical ones at swarm energies and never exceed c at high
energies."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import synth
from oracle.tallies import tallies

QE, ME, AMU = oracle.constants()
C = oracle.light_speed()


def _model(E, rel=1, **kw):
    return oracle.OracleModel([synth.maxwell_component(4.0)], E, relativistic=rel, **kw)


def _ode(E, u0, T, B=0.0, th=0.0):
    """du/dt = -(e/m) (E z^ + v x B), dr/dt = v = u / sqrt(1 + u^2/c^2), integrated
    numerically (B in the xz plane at angle th from E)."""
    k = -QE / ME
    Ev = np.array([0.0, 0.0, E])
    Bv = B * np.array([math.sin(th), 0.0, math.cos(th)])

    def f(t, y):
        u = y[3:]
        v = u / math.sqrt(1.0 + u @ u / C ** 2)
        return np.concatenate([v, k * (Ev + np.cross(v, Bv))])

    sol = solve_ivp(f, (0.0, T), np.concatenate([np.zeros(3), u0]), method="DOP853", rtol=1e-12,
                    atol=1e-30)
    return sol.y[:3, -1], sol.y[3:, -1]


@pytest.mark.parametrize("E", [1e5, 3e8, 0.0])
def test_motion_matches_lorentz_force_integration(E):
    m = _model(E)
    rng = np.random.default_rng(2)
    for _ in range(6):
        u0 = rng.normal(size=3) * C * rng.choice([1e-3, 0.3, 3.0])
        speed = np.linalg.norm(u0)
        T = float(rng.uniform(0.2, 3.0) * max(speed / (QE * max(E, 1.0) / ME), 1e-12))
        r, u = m.move(np.zeros(3), u0, T)
        r_ref, u_ref = _ode(E, u0, T)
        np.testing.assert_allclose(u, u_ref, rtol=1e-10, atol=1e-9 * speed)
        np.testing.assert_allclose(r, r_ref, rtol=1e-9, atol=1e-9 * np.abs(r_ref).max())


@pytest.mark.parametrize("E,B,th", [(1e5, 0.5, 0.7), (3e8, 2.0, 1.2), (0.0, 1.0, 0.3), (2e4, 1.0, math.pi / 2),
                                    (3e8, 1.0, math.pi / 2), (1e3, 3.0, 0.0)])
def test_crossed_fields_match_lorentz_force_integration(E, B, th):
    # (3e8 V/m, 1 T, crossed: |E| = c|B|, the degenerate case of the field invariants)
    m = _model(E, B_T=B, B_angle_rad=th)
    rng = np.random.default_rng(int(E) % 97 + int(B * 10))
    for _ in range(5):
        u0 = rng.normal(size=3) * C * rng.choice([1e-3, 0.5, 3.0])
        T = float(rng.uniform(0.3, 3.0) / (QE * B / ME))
        r, u = m.move(np.zeros(3), u0, T)
        r_ref, u_ref = _ode(E, u0, T, B, th)
        np.testing.assert_allclose(u, u_ref, rtol=0, atol=1e-11 * np.abs(u_ref).max())
        np.testing.assert_allclose(r, r_ref, rtol=0, atol=1e-11 * np.abs(r_ref).max())


@pytest.mark.parametrize("T", [3e-8, 1e-6])
def test_long_flight_in_strong_oblique_field(T):
    # gamma grows like exp(l tau) in proper time: a first guess tau = T is hundreds of e-folds
    # too far, and the proper time must still be found
    E, B, th = 3e7, 0.05, 0.4
    m = _model(E, B_T=B, B_angle_rad=th)
    u0 = np.array([3e5, -1e5, 2e5])
    r, u = m.move(np.zeros(3), u0, T)
    r_ref, u_ref = _ode(E, u0, T, B, th)
    np.testing.assert_allclose(u, u_ref, rtol=0, atol=1e-10 * np.abs(u_ref).max())
    np.testing.assert_allclose(r, r_ref, rtol=0, atol=1e-10 * np.abs(r_ref).max())
    assert math.sqrt(1 + u @ u / C ** 2) > 100


def test_relativistic_cyclotron_period():
    # E = 0: gamma is constant and the transverse motion closes after T = 2 pi gamma m / (e B)
    B = 1.5
    m = _model(0.0, B_T=B, B_angle_rad=0.0)
    for beta_gamma in (1e-3, 0.7, 5.0):
        u0 = np.array([beta_gamma * C, 0.0, 0.2 * beta_gamma * C])
        g = math.sqrt(1 + u0 @ u0 / C ** 2)
        T = 2 * math.pi * g * ME / (QE * B)
        r, u = m.move(np.zeros(3), u0, T)
        np.testing.assert_allclose(u, u0, rtol=0, atol=1e-12 * np.linalg.norm(u0))
        assert abs(r[0]) < 1e-11 * np.linalg.norm(r) and abs(r[1]) < 1e-11 * np.linalg.norm(r)
        assert r[2] == pytest.approx(u0[2] / g * T, rel=1e-12)


def test_crossed_fields_classical_limit_and_work():
    E, B, th = 2e4, 0.8, 1.0
    rel, cl = _model(E, 1, B_T=B, B_angle_rad=th), _model(E, 0, B_T=B, B_angle_rad=th)
    u0 = np.array([2e5, -1e5, 3e5])
    for T in (1e-13, 1e-11, 3e-11):
        r1, u1 = rel.move(np.zeros(3), u0, T)
        r0, v0 = cl.move(np.zeros(3), u0, T)
        beta2 = max(u0 @ u0, u1 @ u1) / C ** 2
        np.testing.assert_allclose(r1, r0, rtol=0, atol=10 * beta2 * np.abs(r0).max())
        # the magnetic force does no work: the energy gain is the work of E alone
        assert rel.kinetic(u1) - rel.kinetic(u0) == pytest.approx(-E * r1[2], rel=1e-9)
    # B -> 0 joins the uniform-E closed form
    tiny, none = _model(E, B_T=1e-12), _model(E)
    r1, u1 = tiny.move(np.zeros(3), u0, 1e-11)
    r2, u2 = none.move(np.zeros(3), u0, 1e-11)
    np.testing.assert_allclose(r1, r2, rtol=1e-9)


def test_hyperbolic_motion_from_rest():
    E = 2e6
    m = _model(E)
    a = -QE * E / ME
    for T in (1e-15, 1e-12, 1e-9, 1e-6):
        r, u = m.move(np.zeros(3), np.zeros(3), T)
        z = C ** 2 / a * (math.sqrt(1.0 + (a * T / C) ** 2) - 1.0)
        assert r[2] == pytest.approx(z, rel=1e-9)
        assert r[0] == 0.0 and r[1] == 0.0
        # speed below c, approaching it
        v = np.linalg.norm(u) / math.sqrt(1.0 + u @ u / C ** 2)
        assert v < C


def test_classical_limit():
    E = 1e4
    rel, cl = _model(E, 1), _model(E, 0)
    u0 = np.array([2e5, -1e5, 3e5])
    for T in (1e-13, 1e-11, 1e-9):
        r1, u1 = rel.move(np.zeros(3), u0, T)
        r0, v0 = cl.move(np.zeros(3), u0, T)
        beta2 = max(u0 @ u0, u1 @ u1) / C ** 2
        np.testing.assert_allclose(r1, r0, rtol=4 * beta2, atol=0)
        np.testing.assert_allclose(u1, v0, rtol=1e-12)


@pytest.mark.parametrize("E", [1e5, 1e8])
def test_work_energy_theorem(E):
    m = _model(E)
    rng = np.random.default_rng(7)
    for _ in range(20):
        u0 = rng.normal(size=3) * C * 0.5
        T = float(rng.uniform(1e-14, 1e-10))
        r, u = m.move(np.zeros(3), u0, T)
        gain = m.kinetic(u) - m.kinetic(u0)
        work = -E * r[2]            # (charge -e) x E x dz, in eV
        assert gain == pytest.approx(work, rel=1e-9, abs=1e-12 * m.kinetic(u0))


def test_speed_at_rest_energy_and_limits():
    m = _model(1e5)
    mc2 = ME * C ** 2 / QE
    # gamma = 2 at eps = m c^2: v = c sqrt(3)/2, u = gamma v = c sqrt(3)
    assert m.speed(mc2) == pytest.approx(C * math.sqrt(3) / 2, rel=1e-14)
    assert m.speed(mc2, proper=True) == pytest.approx(C * math.sqrt(3), rel=1e-14)
    for eps in (1e-3, 1.0, 1e3, 1e6, 1e9):
        assert m.speed(eps) < C
        assert m.kinetic([0.0, 0.0, m.speed(eps, proper=True)]) == pytest.approx(eps, rel=1e-13)
    # classical limit of the rate factor
    assert m.speed(0.01) == pytest.approx(math.sqrt(2 * 0.01 * QE / ME), rel=1e-7)
    cl = _model(1e5, 0)
    assert cl.speed(mc2) == pytest.approx(math.sqrt(2 * mc2 * QE / ME), rel=1e-14)


def test_swarm_matches_classical_at_swarm_energies():
    cfg = synth.cfg1_maxwell(n_electrons=4000, n_collisions=3000)
    a = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 1).records)
    b = tallies(oracle.OracleModel.from_config(cfg.scaled(relativistic=1)).run(cfg.n_electrons, cfg.n_collisions,
                                                                               1).records)
    for key in ("W", "mean_energy", "D"):
        assert abs(a[key][0] - b[key][0]) < 3 * math.hypot(a[key][1], b[key][1]) + 1e-4 * abs(a[key][0]), key


def test_fast_electrons_stay_below_c():
    # a weakly colliding gas in a strong field: keV to MeV electrons
    comp = synth.maxwell_component(4.0, k=synth.tables.MAXWELL_K * 1e-3, min_exp2=-14, max_exp2=24)
    cfg = synth.SwarmConfig([comp], 3e7, init_energy_eV=1.0, n_electrons=200, n_collisions=300,
                            relativistic=1)
    m = oracle.OracleModel.from_config(cfg, grid_emax=24)
    r = m.run(200, 300, 3).records
    dist = np.linalg.norm(r["r"], axis=1)
    assert np.all(dist / r["t"] < C)
    assert np.max(r["sum_eps"] / 300) > 1e4      # relativistic energies reached
    c = oracle.OracleModel.from_config(cfg.scaled(relativistic=0), grid_emax=24).run(200, 300, 3).records
    assert np.max(np.linalg.norm(c["r"], axis=1) / c["t"]) > C   # the classical mover would not


def test_crossed_field_swarm_matches_classical():
    cfg = synth.cfg1_maxwell(n_electrons=1500, n_collisions=1000).scaled(B_T=2.0, B_angle_rad=math.pi / 4)
    a = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 1).records)
    b = tallies(oracle.OracleModel.from_config(cfg.scaled(relativistic=1)).run(cfg.n_electrons, cfg.n_collisions,
                                                                               1).records)
    for key in ("W", "Wx", "Wy", "mean_energy"):
        assert abs(a[key][0] - b[key][0]) < 3 * math.hypot(a[key][1], b[key][1]) + 1e-4 * abs(a[key][0]), key


def test_invalid_relativistic_refused():
    with pytest.raises(ValueError):
        oracle.OracleModel.from_config(synth.cfg1_maxwell().scaled(relativistic=1, thermal_targets=1))
    with pytest.raises(ValueError):
        oracle.OracleModel.from_config(synth.cfg1_maxwell().scaled(relativistic=2))
