"""Pins of the oracle's moving targets (section "Effect of gas temperature": the target
velocity from the Maxwell-Boltzmann distribution of the gas, and the paper's equation for the
electron's velocity after the collision in the centre-of-momentum frame).

  * the target velocity: three independent normals of spread sqrt(kT/M) (Kolmogorov-Smirnov);
  * the electron's new velocity with the paper's second equation (the target's) conserves
    momentum and, less the threshold energy, kinetic energy;
  * with the target at rest it reduces to eqs. delta_energy_ela and delta_energy_ine with
    theta the centre-of-momentum angle;
  * a process below its threshold in the centre-of-momentum frame cannot happen;
  * without a field the mean energy per collision relaxes to (3/2) kT exactly as
    E[eps'] = (1 - kappa) eps + kappa (3/2) kT, kappa = 2 m M / (m + M)^2, predicts for any
    cross-section, and the same holds for the mean energy after the collisions;
  * at a high field the moving targets change nothing measurable; at a very low field they
    keep the swarm at the gas temperature instead of letting it cool below it.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from oracle.tallies import tallies

QE, ME, AMU = oracle.constants()
KB = oracle.boltzmann()


def test_target_velocity_is_maxwell_boltzmann():
    sigma = 1234.5
    rng = np.random.default_rng(5)
    v = np.array([oracle.target_velocity(sigma, rng.random(4)) for _ in range(20000)])
    for i in range(3):
        assert stats.kstest(v[:, i] / sigma, "norm").pvalue > 1e-3
    # the three components are uncorrelated, and independent: |V|^2 / sigma^2 is chi-square
    # with three degrees of freedom
    c = np.corrcoef(v.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 0.03)
    assert stats.kstest((v * v).sum(axis=1) / sigma ** 2, stats.chi2(3).cdf).pvalue > 1e-3


@pytest.mark.parametrize("M_amu,eps_k", [(4.0, 0.0), (40.0, 11.5), (1.0, 3.0), (200.0, 0.08)])
def test_moving_target_conserves_momentum_and_energy(M_amu, eps_k):
    rng = np.random.default_rng(int(M_amu * 10 + eps_k))
    m, M = ME, M_amu * AMU
    n_ok = 0
    for _ in range(200):
        V1 = rng.normal(size=3) * 3e6
        V2 = rng.normal(size=3) * 400.0
        uh = rng.normal(size=3)
        uh /= np.linalg.norm(uh)
        V1p = oracle.moving_target(V1, V2, M_amu, eps_k, uh)
        Vcm = (m * V1 + M * V2) / (m + M)
        arg2 = np.dot(V2 - Vcm, V2 - Vcm) - 2 * eps_k * QE / (m + M) * (m / M)
        if V1p is None:
            # below the threshold in the centre-of-momentum frame
            assert 0.5 * m * M / (m + M) * np.dot(V1 - V2, V1 - V2) < eps_k * QE * (1 + 1e-12)
            continue
        n_ok += 1
        V2p = Vcm - math.sqrt(arg2) * uh          # the paper's equation for the target
        p0, p1 = m * V1 + M * V2, m * V1p + M * V2p
        np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-12 * np.linalg.norm(p0))
        e0 = 0.5 * m * V1 @ V1 + 0.5 * M * V2 @ V2
        e1 = 0.5 * m * V1p @ V1p + 0.5 * M * V2p @ V2p + eps_k * QE
        assert abs(e1 - e0) < 1e-11 * e0
    assert n_ok > 150


@pytest.mark.parametrize("M_amu,eps_k", [(40.0, 0.0), (4.0, 0.0), (40.0, 11.5), (44.0, 0.3)])
def test_target_at_rest_reduces_to_energy_transfer_equations(M_amu, eps_k):
    rng = np.random.default_rng(3)
    kind = synth.ELASTIC if eps_k == 0 else synth.EXCITATION
    for _ in range(100):
        eps = eps_k * 1.5 + rng.uniform(0.1, 50.0)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        V1 = d * math.sqrt(2 * eps * QE / ME)
        uh = rng.normal(size=3)
        uh /= np.linalg.norm(uh)
        V1p = oracle.moving_target(V1, np.zeros(3), M_amu, eps_k, uh)
        epsp = 0.5 * ME * V1p @ V1p / QE
        # theta = the angle in the centre-of-momentum frame, measured from V1 (V2 = 0)
        want = oracle.energy_after(kind, eps, eps_k, float(uh @ d), M_amu)
        assert epsp == pytest.approx(want, rel=1e-10, abs=1e-14 * eps)


def test_below_threshold_in_cm_frame_is_forbidden():
    # a 1 eV electron cannot excite a 2 eV level, whatever the target's thermal speed
    V1 = np.array([0.0, 0.0, math.sqrt(2 * 1.0 * QE / ME)])
    assert oracle.moving_target(V1, np.array([300.0, 0.0, -200.0]), 40.0, 2.0, [1.0, 0.0, 0.0]) is None
    assert oracle.moving_target(V1, np.zeros(3), 40.0, 0.99, [1.0, 0.0, 0.0]) is not None


def _relaxation(eps0, T, M_amu, n, comp=None):
    comp = comp or synth.maxwell_component(M_amu)
    cfg = synth.SwarmConfig([comp], 0.0, init_energy_eV=eps0, T_K=T, thermal_targets=1,
                            n_electrons=4000, n_collisions=n)
    Tl = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 7).records)
    M = M_amu * AMU
    kappa = 2 * ME * M / (ME + M) ** 2
    eth = 1.5 * KB * T / QE
    # mean over the n collisions of E[eps_j] = eth + (eps0 - eth)(1 - kappa)^j, j = 0..n-1
    mean = eth + (eps0 - eth) * (1 - (1 - kappa) ** n) / (n * kappa)
    mean_after = (1 - kappa) * mean + kappa * eth
    return Tl, mean, mean_after


@pytest.mark.parametrize("eps0,T,M_amu,n", [(1.0, 293.0, 1.0, 3000), (0.001, 293.0, 4.0, 2000),
                                           (0.5, 2000.0, 2.0, 1500), (0.2, 0.0, 1.0, 1000)])
def test_zero_field_relaxation_closed_form(eps0, T, M_amu, n):
    T_, mean, mean_after = _relaxation(eps0, T, M_amu, n)
    for key, want in (("mean_energy", mean), ("mean_energy_after", mean_after)):
        v, sig, _ = T_[key]
        assert abs(v - want) < 4 * sig + 1e-9 * want, (key, v, want, sig)


def test_zero_field_relaxation_any_cross_section():
    # an argon-like elastic table (energy-dependent rate): the closed form still holds
    comp = synth.cfg2_argon_sweep()[0].components[0]
    comp = synth.Component(2.0, 1.0, [ch for ch in comp.channels if ch.kind == synth.ELASTIC])
    T_, mean, _ = _relaxation(0.6, 600.0, 2.0, 1500, comp)
    v, sig, _ = T_["mean_energy"]
    assert abs(v - mean) < 4 * sig, (v, mean, sig)


def test_high_field_unchanged_low_field_held_at_gas_temperature():
    sweep = synth.cfg2_argon_sweep(n_electrons=1500, n_collisions=1500)
    cfg = sweep[21]
    a = tallies(oracle.OracleModel.from_config(cfg).run(1500, 1500, 2).records)
    b = tallies(oracle.OracleModel.from_config(cfg.scaled(thermal_targets=1)).run(1500, 1500, 2).records)
    for key in ("W", "mean_energy"):
        assert abs(a[key][0] - b[key][0]) < 4 * math.hypot(a[key][1], b[key][1]) + 0.01 * abs(a[key][0])
    # 1e-3 Td with 0.001 eV primaries: at rest the swarm stays far below kT; moving targets
    # heat it towards (3/2) kT = 0.038 eV (argon's relaxation takes 1/kappa ~ 3.7e4 collisions)
    low = cfg.scaled(E_V_per_m=synth.td_to_field(1e-3), init_energy_eV=0.001)
    c = tallies(oracle.OracleModel.from_config(low).run(150, 40000, 2).records)
    d = tallies(oracle.OracleModel.from_config(low.scaled(thermal_targets=1)).run(150, 40000, 2).records)
    eth = 1.5 * KB * 293.0 / QE
    assert c["mean_energy"][0] < 0.1 * eth
    assert d["mean_energy"][0] > 0.3 * eth and d["mean_energy"][0] > 5 * c["mean_energy"][0]


def _threshold_gas(T_K, thermal):
    """A 1-u gas with a Maxwell elastic channel and a 0.05 eV excitation, in a weak field."""
    el = synth.maxwell_component(1.0).channels[0]
    e = np.geomspace(0.05, 1000.0, 200)
    exc = synth.Channel(synth.EXCITATION, 0.05, e, np.full(len(e), 2e-20))
    comp = synth.Component(1.0, 1.0, [el, exc])
    return synth.SwarmConfig([comp], synth.td_to_field(0.3), init_energy_eV=0.06, T_K=T_K,
                             thermal_targets=thermal)


def test_threshold_decided_in_cm_frame():
    """With moving targets the threshold applies in the centre-of-momentum frame: excitations
    happen below the laboratory onset eps_k (m+M)/M (target moving towards the electron) and
    candidates above it are forbidden (target moving away).  With targets at rest neither
    happens."""
    onset = 0.05 * (ME + AMU) / AMU
    ids = list(range(64))
    found = {}
    for thermal in (0, 1):
        cfg = _threshold_gas(3000.0, thermal)
        ev = oracle.OracleModel.from_config(cfg).run(64, 1500, 4, trace_ids=ids, max_events=2048).events
        real_exc = ev[(ev["type"] == oracle.EV_REAL) & (ev["channel"] == 1)]
        forb = ev[ev["type"] == oracle.EV_FORBIDDEN]
        found[thermal] = (int((real_exc["eps"] < onset).sum()), int((forb["eps"] >= onset).sum()),
                          len(real_exc), len(forb))
    assert found[0][0] == 0 and found[0][1] == 0 and found[0][2] > 0
    assert found[1][0] > 0 and found[1][1] > 0, found


def test_invalid_temperature_refused():
    cfg = synth.cfg1_maxwell().scaled(thermal_targets=1, T_K=-1.0)
    with pytest.raises(ValueError):
        oracle.OracleModel.from_config(cfg)
