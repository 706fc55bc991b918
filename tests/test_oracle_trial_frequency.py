"""Pins of the oracle's variable trial frequency (section "Trial frequency strategies": the
VariableTrialFrequency nu' = (1 + zeta) nu(eps), kept for a grace number of trials, with a
return to the last real collision when nu(eps) > nu' is found).

Exact special cases:
  * nu' is capped at the constant strategy's value, so a huge zeta gives records equal, bit
    for bit, to the constant-frequency run (same streams, same decisions);
  * a constant-rate gas never fails, its efficiency is 1/(1+zeta) (binomial), and the drift
    velocity and mean energy keep their closed forms eE/(m nu) and the Maxwell value;
  * without a field and with infinitely heavy targets the energy of every electron is
    constant, so no trial can fail whatever zeta and grace are.
Statistical: on the argon-like gas the tallies agree with the exact constant-frequency
method, with a higher efficiency, and fails do occur.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies

QE, ME, AMU = oracle.constants()


def _variable(cfg, **kw):
    return cfg.scaled(trial_strategy=1, **kw)


def test_capped_variable_equals_constant_bitwise():
    cfg = synth.cfg2_argon_sweep(n_electrons=150, n_collisions=600)[15]
    a = oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 3).records
    b = oracle.OracleModel.from_config(_variable(cfg, trial_zeta=1e30, trial_grace=7)).run(
        cfg.n_electrons, cfg.n_collisions, 3).records
    assert a.tobytes() == b.tobytes()
    assert int(b["n_fail"].sum()) == 0


@pytest.mark.parametrize("zeta", [0.25, 1.0])
def test_constant_rate_gas_efficiency_and_closed_forms(zeta):
    # nu = 1e12 at every energy; the constant strategy's nu' is fixed at 4e12 (the cap), so
    # the variable strategy runs at nu' = (1 + zeta) 1e12 and accepts a trial with
    # probability 1/(1 + zeta).
    cfg = synth.cfg1_maxwell(n_electrons=3000, n_collisions=2000).scaled(
        user_majorant=4e12, trial_strategy=1, trial_zeta=zeta, trial_grace=50)
    r = oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 1)
    T = tallies(r.records)
    assert T["n_fail"] == 0 and T["n_forbidden"] == 0
    trials = T["n_real"] + T["n_null"]
    p = 1.0 / (1.0 + zeta)
    assert abs(T["efficiency"] - p) < 4.5 * math.sqrt(p * (1 - p) / trials)
    W = QE * synth.td_to_field(10.0) / (ME * 1e12)
    assert abs(T["W"][0] - W) < 3.5 * T["W"][1]
    # mean energy before a collision, averaged over the n collisions: isotropic restarts
    # give E[eps'] = (1 - kappa) eps and a mean flight gain m W^2, so the sequence relaxes
    # geometrically from eps0 + m W^2 towards m W^2 / kappa
    M = 4.0 * AMU
    kappa = 2 * ME * M / (ME + M) ** 2
    delta = ME * W * W / QE
    n = cfg.n_collisions
    xs, x1 = delta / kappa, cfg.init_energy_eV + delta
    mean = xs + (x1 - xs) * (1 - (1 - kappa) ** n) / (n * kappa)
    assert abs(T["mean_energy"][0] - mean) < 3.5 * T["mean_energy"][1]


def test_no_field_heavy_targets_never_fail():
    # E = 0 and an elastic channel on a 1e12-u target: eps is constant between and (up to
    # 2m/M ~ 1e-15) across collisions, so nu(eps) <= (1 + zeta) nu(eps_0) always holds.
    comp = synth.random_component(np.random.default_rng(9), fraction=1.0, max_inelastic=0)
    comp = synth.Component(1e12, 1.0, [ch for ch in comp.channels if ch.kind == synth.ELASTIC])
    cfg = synth.SwarmConfig([comp], 0.0, init_energy_eV=3.0, n_electrons=400, n_collisions=500,
                            trial_strategy=1, trial_zeta=0.05, trial_grace=1)
    T = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 2).records)
    assert T["n_fail"] == 0
    assert T["efficiency"] > 0.9


@pytest.fixture(scope="module")
def argon_pair():
    cfg = synth.cfg2_argon_sweep(n_electrons=3000, n_collisions=3000)[10]
    a = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 0).records)
    v = tallies(oracle.OracleModel.from_config(_variable(cfg)).run(
        cfg.n_electrons, cfg.n_collisions, 0).records)
    return a, v


def test_variable_matches_exact_method_on_argon(argon_pair):
    a, v = argon_pair
    for key in ("W", "mean_energy", "D", "DL", "DT"):
        va, sa, _ = a[key]
        vb, sb, _ = v[key]
        assert abs(va - vb) <= 3.5 * math.hypot(sa, sb) + 0.005 * abs(va), (key, va, vb, sa, sb)


def test_variable_is_more_efficient_and_fails(argon_pair):
    a, v = argon_pair
    assert v["n_real"] == a["n_real"]
    assert v["efficiency"] > 2.0 * a["efficiency"], (v["efficiency"], a["efficiency"])
    assert v["n_fail"] > 0
    trials = v["n_real"] + v["n_null"] + v["n_forbidden"] + v["n_fail"]
    assert abs(v["efficiency"] - v["n_real"] / trials) < 1e-15
