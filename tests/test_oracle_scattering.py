"""Pins of the oracle's anisotropic scattering (section "Theoretical framework", eqs.
collision_angle and collision_angle_xi, after Okhrimovskyy et al.) against mathematics that
does not use its code: quadrature of the sampled cos(theta) over the uniform, the Taylor
series of the xi relation, the algebraic identity between the atomic and the xi forms,
spherical coordinates for the rotation, and the Maxwell-gas drift velocity eE/(m nu_m) with
the momentum-transfer frequency nu_m = nu (1 - <cos theta>)."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from oracle.tallies import tallies

QE, ME, AMU = oracle.constants()


@pytest.mark.parametrize("r", [0.9, 0.5, 0.2, 0.05])
def test_xi_form_mean_momentum_transfer_equals_ratio(r):
    # The xi equation says sigma_mt/sigma_el = <1 - cos theta> of the xi distribution:
    # integrate 1 - cos(theta(u)) over u with the sampling formula itself.
    xi = oracle.xi_from_ratio(r)
    assert 0.0 < xi < 1.0
    val, err = integrate.quad(lambda u: 1.0 - oracle.scatter_cos(2, xi, 1.0, u), 0.0, 1.0,
                              epsabs=1e-13, epsrel=1e-12, limit=200)
    assert abs(val - r) < 1e-9, (r, xi, val)


def test_xi_relation_series_and_limits():
    # with ln((1+x)/(1-x)) = 2 sum x^(2k+1)/(2k+1):
    # (1-x)/(2x^2) ((1+x) ln((1+x)/(1-x)) - 2x) = 1 - 2x/3 - 2x^3/15 - 2x^5/35 - ...
    for x in (1e-3, 1e-2, 3e-2, 0.1):
        series = 1 - 2 * x / 3 - 2 * x ** 3 / 15 - 2 * x ** 5 / 35
        # (the closed form cancels: its rounding error grows like 1e-16 / x^2)
        assert abs(oracle.mt_over_el_of_xi(x) - series) < x ** 7 + 1e-16 / x ** 2
    assert oracle.mt_over_el_of_xi(0.0) == 1.0
    assert oracle.mt_over_el_of_xi(1 - 1e-9) < 1e-7
    assert oracle.xi_from_ratio(1.0) == 0.0
    # isotropic limit of the xi form: cos = 1 - 2u
    for u in (0.0, 0.3, 0.77):
        assert oracle.scatter_cos(2, 0.0, 5.0, u) == 1.0 - 2.0 * u


@pytest.mark.parametrize("eps", [0.01, 1.0, 15.0, 300.0])
def test_screened_coulomb_mean_and_identity(eps):
    e = eps / oracle.hartree_eV()
    a = 8.0 * e
    # <1 - cos> = int_0^1 2u/(1 + a(1-u)) du = 2(-1/a + (1 + 1/a) ln(1 + a)/a)
    closed = 2.0 * (-1.0 / a + (1.0 + 1.0 / a) * math.log1p(a) / a)
    val, _ = integrate.quad(lambda u: 1.0 - oracle.scatter_cos(1, 0.0, eps, u), 0.0, 1.0,
                            epsabs=1e-13, epsrel=1e-12)
    assert abs(val - closed) < 1e-9 * max(1.0, closed)
    # the atomic form is the xi form with xi = 4e/(1 + 4e)
    xi = 4 * e / (1 + 4 * e)
    for u in np.linspace(0.0, 0.999, 7):
        assert abs(oracle.scatter_cos(1, 0.0, eps, u) - oracle.scatter_cos(2, xi, 0.0, u)) < 1e-12
    # very low energy: nearly isotropic
    assert abs(oracle.scatter_cos(1, 0.0, 1e-9, 0.25) - 0.5) < 1e-8


def test_rotation_geometry():
    rng = np.random.default_rng(4)
    for _ in range(200):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = rng.uniform(-1, 1)
        phi = rng.uniform(0, 2 * math.pi)
        n = oracle.rotate(d, c, phi)
        assert abs(np.linalg.norm(n) - 1) < 1e-13
        assert abs(n @ d - c) < 1e-13
        # opposite azimuths mirror the perpendicular part
        m = oracle.rotate(d, c, phi + math.pi)
        np.testing.assert_allclose((n - c * d) + (m - c * d), 0.0, atol=1e-13)
    # along z: spherical coordinates (sin cos phi, sin sin phi, cos)
    c, phi = 0.3, 1.1
    s = math.sqrt(1 - c * c)
    np.testing.assert_allclose(oracle.rotate([0, 0, 1], c, phi), [s * math.cos(phi), s * math.sin(phi), c],
                               atol=1e-15)
    # azimuth uniform about d: the mean perpendicular part over phi vanishes
    d = np.array([0.6, -0.48, 0.64])
    ps = np.linspace(0, 2 * math.pi, 64, endpoint=False)
    mean = np.mean([oracle.rotate(d, 0.2, p) for p in ps], axis=0)
    np.testing.assert_allclose(mean, 0.2 * d, atol=1e-13)


@pytest.mark.parametrize("r", [1.0, 0.5, 0.25])
def test_maxwell_gas_drift_with_anisotropic_scattering(r):
    # Constant collision frequency nu and energy-independent <1 - cos theta> = r: momentum
    # balance gives W = eE/(m nu r) (the recoil correction is of order m/M ~ 1e-4).
    comp = synth.maxwell_component(4.0).with_scattering(2 if r < 1 else 0, r)
    cfg = synth.SwarmConfig([comp], synth.td_to_field(10.0), n_electrons=6000, n_collisions=6000)
    T = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 3).records)
    W = QE * synth.td_to_field(10.0) / (ME * 1e12 * r)
    assert abs(T["W"][0] - W) < 3.5 * T["W"][1] + 2e-3 * W, (T["W"], W)
    assert abs(T["Wx"][0]) < 4 * T["Wx"][1] and abs(T["Wy"][0]) < 4 * T["Wy"][1]


def test_screened_coulomb_changes_argon_transport():
    # Forward scattering lowers the momentum-transfer rate: faster drift than isotropic.
    cfg = synth.cfg2_argon_sweep(n_electrons=2000, n_collisions=2000)[21]
    a = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 1).records)
    comps = [c.with_scattering(1) for c in cfg.components]
    b = tallies(oracle.OracleModel.from_config(cfg.scaled(components=comps)).run(
        cfg.n_electrons, cfg.n_collisions, 1).records)
    assert b["W"][0] > a["W"][0] + 3 * math.hypot(a["W"][1], b["W"][1])


def test_invalid_scattering_refused():
    comp = synth.maxwell_component(4.0).with_scattering(2, 1.5)
    with pytest.raises(ValueError):
        oracle.OracleModel([comp], 1e5)
    with pytest.raises(ValueError):
        oracle.OracleModel([synth.maxwell_component(4.0).with_scattering(3)], 1e5)
