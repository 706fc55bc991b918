"""Closed-form pins of the whole oracle simulation and its tallies (section 'Determination
of swarm attributes'), on gases where the answer is known exactly."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies

QE, ME, AMU = oracle.constants()
N = 2.5e25


def _within(val, want, sig, k=3.5, rel=0.0):
    assert abs(val - want) <= k * sig + rel * abs(want), (val, want, sig)


@pytest.fixture(scope="module")
def maxwell_run():
    cfg = synth.cfg1_maxwell(n_electrons=8000)
    m = oracle.OracleModel.from_config(cfg)
    r = m.run(cfg.n_electrons, cfg.n_collisions, 0)
    return m, tallies(r.records)


def test_maxwell_drift_velocity(maxwell_run):
    # nu = 1e12 s^-1 at every energy, so W = eE/(m nu) exactly
    m, T = maxwell_run
    W = QE * synth.td_to_field(10.0) / (ME * 1e12)
    assert abs(W - 4.39705e4) < 1.0
    _within(T["W"][0], W, T["W"][1])
    _within(T["Wx"][0], 0.0, T["Wx"][1])
    _within(T["Wy"][0], 0.0, T["Wy"][1])
    assert T["n_stuck"] == 0 and T["n_over"] == 0
    assert T["efficiency"] > 0.999


def test_maxwell_mean_energy(maxwell_run):
    # isotropic restarts: E[eps'] = (1-kappa) eps, flight gain delta = m W^2 (eV):
    # x_i = x* + (x_1 - x*)(1-kappa)^(i-1), x* = delta/kappa, x_1 = eps0 + delta
    m, T = maxwell_run
    M = 4.0 * AMU
    kappa = 2 * ME * M / (ME + M) ** 2
    W = QE * synth.td_to_field(10.0) / (ME * 1e12)
    delta = ME * W * W / QE
    n = 10_000
    xs = delta / kappa
    x1 = 0.1 + delta
    mean = xs + (x1 - xs) * (1 - (1 - kappa) ** n) / (n * kappa)
    assert abs(mean - 26.448) < 2e-3
    _within(T["mean_energy"][0], mean, T["mean_energy"][1])
    _within(T["mean_energy_after"][0], (1 - kappa) * mean, T["mean_energy_after"][1])
    assert T["mean_energy_after"][0] < T["mean_energy"][0]


def test_maxwell_drude_drift_with_crossed_B():
    # nu W = a + omega b x W (Drude) for constant nu; B = 1 T at 45 degrees to E
    E, B, ang = synth.td_to_field(10.0), 1.0, math.pi / 4
    cfg = synth.cfg1_maxwell(n_electrons=6000)
    m = oracle.OracleModel([synth.maxwell_component(4.0)], E, B, ang)
    T = tallies(m.run(cfg.n_electrons, cfg.n_collisions, 0).records)
    nu, om = 1e12, QE * B / ME
    b = np.array([math.sin(ang), 0, math.cos(ang)])
    a = np.array([0, 0, -QE * E / ME])
    bx = np.array([[0, -b[2], b[1]], [b[2], 0, -b[0]], [-b[1], b[0], 0]])
    W = np.linalg.solve(nu * np.eye(3) - om * bx, a)
    np.testing.assert_allclose(W, [-659.7, 5304.4, -43310.8], atol=0.5)
    for i, k in enumerate(("Wx", "Wy", "Wz")):
        _within(T[k][0], W[i], T[k][1])


def test_diffusion_closed_form_no_field():
    # E = 0, very heavy target (no energy loss), constant nu, speed v0: with n real
    # collisions E[D] = 2 v0^2 n / (nu (n+1)), E[D_L] = E[D_T] = v0^2 n / (3 nu (n+1))
    k = synth.tables.MAXWELL_K
    comp = synth.constant_rate_component(1e9, 1.0, k)
    m = oracle.OracleModel([comp], 0.0, init_energy_eV=1.0)
    n, ne = 50, 40000
    T = tallies(m.run(ne, n, 3).records)
    nu = 1e12
    v0 = math.sqrt(2 * QE / ME)
    D = 2 * v0 ** 2 * n / (nu * (n + 1))
    _within(T["D"][0], D, T["D"][1])
    _within(T["DL"][0], D / 6, T["DL"][1])
    _within(T["DT"][0], D / 6, T["DT"][1])
    # the spread across particles is chi-square like with 3, 1, 2 degrees of freedom;
    # the worked example prints +-/mean of about 0.87, 1.25, 1.00 for D, D_L, D_T
    assert abs(T["D"][2] / T["D"][0] - math.sqrt(2 / 3)) < 0.08
    assert abs(T["DL"][2] / T["DL"][0] - math.sqrt(2)) < 0.12
    assert abs(T["DT"][2] / T["DT"][0] - 1.0) < 0.08


def test_spread_tallies_against_independent_random_walk():
    # E = 0, very heavy target, constant nu, speed v0: after n real collisions an electron
    # has made n isotropic, independent steps of length v0 tau, tau ~ Exp(nu) (null
    # collisions thin a Poisson process and turn nothing).  The spread tallies sigma =
    # <2|d|>, sigma_L = <2|d_z|>, sigma_T = <2|d_perp|> (section "Determination of swarm
    # attributes") must equal those of a plain numpy walk of that process, and approach the
    # Gaussian limits E|d| = sqrt(8 <d^2> / (3 pi)), E|d_z| = sqrt(2 <d_z^2> / pi),
    # E|d_perp| = sqrt(pi <d_perp^2> / 4) with <d^2> = 2 n (v0/nu)^2.
    k = synth.tables.MAXWELL_K
    comp = synth.constant_rate_component(1e9, 1.0, k)
    m = oracle.OracleModel([comp], 0.0, init_energy_eV=1.0)
    n, ne = 50, 40000
    T = tallies(m.run(ne, n, 5).records)
    nu, v0 = 1e12, math.sqrt(2 * QE / ME)
    rng = np.random.default_rng(123)
    nw = 400_000
    d = np.zeros((nw, 3))
    for _ in range(n):
        cz = rng.uniform(-1.0, 1.0, nw)
        ph = rng.uniform(0.0, 2 * math.pi, nw)
        sz = np.sqrt(1.0 - cz * cz)
        step = rng.exponential(v0 / nu, nw)
        d[:, 0] += step * sz * np.cos(ph)
        d[:, 1] += step * sz * np.sin(ph)
        d[:, 2] += step * cz
    walk = {"sigma": 2 * np.linalg.norm(d, axis=1), "sigmaL": 2 * np.abs(d[:, 2]),
            "sigmaT": 2 * np.linalg.norm(d[:, :2], axis=1)}
    for key, x in walk.items():
        _within(T[key][0], x.mean(), math.hypot(T[key][1], x.std() / math.sqrt(nw)), k=4.0)
    d2 = 2 * n * (v0 / nu) ** 2
    gauss = {"sigma": 2 * math.sqrt(8 * d2 / (3 * math.pi)), "sigmaL": 2 * math.sqrt(2 * d2 / (3 * math.pi)),
             "sigmaT": 2 * math.sqrt(math.pi * (2 * d2 / 3) / 4)}
    for key, want in gauss.items():
        assert abs(T[key][0] / want - 1) < 0.03, (key, T[key][0] / want)


def _const_rates(k_el, k_ion, k_att):
    return synth.constant_rate_component(4.0, 1.0, k_el, k_ion, k_att)


def test_townsend_coefficients_constant_rates_dummy():
    # dummy ionisation/attachment: G and D per unit drift length are nu_i/W and nu_a/W
    k = synth.tables.MAXWELL_K
    comp = _const_rates(0.8 * k, 0.15 * k, 0.05 * k)
    E = synth.td_to_field(30.0)
    m = oracle.OracleModel([comp], E)
    T = tallies(m.run(4000, 4000, 11).records)
    nu = 1e12
    W = QE * E / (ME * nu)
    _within(T["W"][0], W, T["W"][1])
    assert abs(T["alpha_rate"] / (0.15 * nu / W) - 1) < 0.02
    assert abs(T["eta_rate"] / (0.05 * nu / W) - 1) < 0.04
    assert T["n_attached"] == 0 and T["n_created"] == 0


def test_real_secondaries_population():
    # lineage budgets: E[#completing] = N0 (1+p-q)^n, E[#attached] = N0 q sum_{k<n} (1+p-q)^k
    k = synth.tables.MAXWELL_K
    p, q = 0.01, 0.005
    comp = _const_rates((1 - p - q) * k, p * k, q * k)
    m = oracle.OracleModel([comp], synth.td_to_field(30.0), secondaries=1)
    n0, n = 3000, 200
    r = m.run(n0, n, 5)
    T = tallies(r.records)
    g = 1 + p - q
    fin = n0 * g ** n
    att = n0 * q * sum(g ** j for j in range(n))
    assert abs(T["n_finished"] / fin - 1) < 0.05
    assert abs(T["n_attached"] / att - 1) < 0.06
    assert T["n_electrons"] == n0 + T["n_created"]
    ids = r.records["id"]
    assert len(np.unique(ids)) == len(ids)
    # every real collision of every electron is counted once: sum over lineage budgets
    kr = r.records["k_end"].astype(np.int64) - r.records["k_start"]
    assert T["n_real"] == int(kr.sum())


def test_capacity_error_is_reported():
    k = synth.tables.MAXWELL_K
    comp = _const_rates(0.8 * k, 0.2 * k, 0.0)
    m = oracle.OracleModel([comp], synth.td_to_field(30.0), secondaries=1)
    r = m.run(10, 200, 1, capacity=50)
    assert r.status == -3


def test_null_collision_invariance():
    # doubling the trial frequency leaves the swarm statistically unchanged and the null
    # fraction becomes 1 - nu/nu'
    cfg = synth.cfg1_maxwell(n_electrons=3000, n_collisions=3000)
    m1 = oracle.OracleModel.from_config(cfg)
    m2 = oracle.OracleModel.from_config(cfg, user_majorant=2e12)
    T1 = tallies(m1.run(3000, 3000, 2).records)
    T2 = tallies(m2.run(3000, 3000, 2).records)
    for key in ("W", "mean_energy", "D"):
        d = abs(T1[key][0] - T2[key][0])
        assert d < 4 * math.hypot(T1[key][1], T2[key][1]), key
    assert abs(T2["efficiency"] - 0.5) < 0.003


def test_worked_example_identities():
    # D = 2 D_L + 4 D_T holds for the printed values and for the estimator definitions
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")))
    assert abs(g["D_cm2_per_s"] - (2 * g["DL_cm2_per_s"] + 4 * g["DT_cm2_per_s"])) < 0.1
    assert g["real"] == g["particles"] * g["interactions"] * g["events"]
    eff = g["real"] / (g["real"] + g["null"] + g["fail"])
    assert abs(100 * eff - g["efficiency_percent"]) < 1e-3
    mu = g["W_cm_per_us"] * 1e6 / (g["field_kV_per_cm"] * 1e3)     # cm^2 / (V s)
    assert abs(mu / g["mu_cm2_per_Vs"] - 1) < 1e-5
    assert abs(g["D_cm2_per_s"] / mu / g["D_over_mu_V"] - 1) < 1e-4
    cfg = synth.cfg1_maxwell(n_electrons=500, n_collisions=2000)
    T = tallies(oracle.OracleModel.from_config(cfg).run(500, 2000, 9).records)
    assert abs(T["D"][0] - (2 * T["DL"][0] + 4 * T["DT"][0])) < 1e-12 * T["D"][0]
