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
Brute force: a plain-Python run of the strategy's steps for a few electrons, built on the
oracle's primitives (streams, motion, rate lookup, channel choice, energy transfer) but not
on its loop, gives the same records, fail counts included, at grace counts from 1 to 300.
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


# ---- brute force ------------------------------------------------------------------------

def _iso(u_cos, u_phi):
    ct = 1.0 - 2.0 * u_cos
    st = math.sqrt(max(0.0, (1.0 - ct) * (1.0 + ct)))
    ph = 2.0 * math.pi * u_phi
    return np.array([st * math.cos(ph), st * math.sin(ph), ct])


def _energy(v):
    return 0.5 * ME * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / QE


def _speed(eps):
    return math.sqrt(2.0 * eps * QE / ME)


def brute_force_variable(m, cfg, zeta, grace0, eid, n_coll, seed):
    """One electron (B = 0, dummy secondaries, isotropic scattering) with the variable trial
    frequency, step by step: nu' = (1 + zeta) nu(eps), capped at the constant value, set
    from the starting energy; every trial spends one of the grace count; a trial finding
    nu(eps) > nu' is a fail: back to the last real collision with nu' from that rate and a
    new grace count; when the count runs out nu' is renewed from the trial's energy (after a
    null or a forbidden pick) or from the energy after the collision."""
    cap = m.majorant

    def renew(eps):
        nu, _ = m.nu_grid(eps)
        return min((1.0 + zeta) * nu, cap)

    h = oracle.stream_block(seed, eid, oracle.INIT_HI, 0)
    l = oracle.stream_block(seed, eid, oracle.INIT_LO, 0)
    v = _iso(oracle.uniform53(h[0], l[0]), oracle.uniform53(h[1], l[1])) * _speed(cfg.init_energy_eV)
    r = np.zeros(3)
    t = 0.0
    T = 0.0
    k = 0
    nup = renew(cfg.init_energy_eV)
    grace = grace0
    rec = dict(n_null=0, n_fail=0, n_forbidden=0, n_over=0, G=0, D=0, sum_eps=0.0, sum_epsp=0.0)
    block = 0
    while k < n_coll:
        hi = oracle.stream_block(seed, eid, oracle.TRIAL_HI, block)
        lo = oracle.stream_block(seed, eid, oracle.TRIAL_LO, block)
        block += 1
        for sub in (0, 1):
            u_f = oracle.uniform53(hi[2 * sub], lo[2 * sub])
            u_r = oracle.uniform53(hi[2 * sub + 1], lo[2 * sub + 1])
            T += -math.log(1.0 - u_f) / nup
            _, vT = m.move(r, v, T)
            eps = _energy(vT)
            nu, over = m.nu_grid(eps)
            if nu > nup:                                   # fail
                rec["n_fail"] += 1
                T = 0.0
                nup = min((1.0 + zeta) * nu, cap)
                grace = grace0
                break
            grace -= 1
            c = m.select(eps, u_r * nup)
            if c < 0:                                      # null
                rec["n_null"] += 1
                if grace == 0:
                    nup, grace = renew(eps), grace0
                continue
            _, kind, thr, mass = m.channel_info[c]
            M = mass * AMU
            if kind in (synth.EXCITATION, synth.IONIZATION) and eps < thr * ((ME + M) / M):
                rec["n_forbidden"] += 1                    # treated as null
                if grace == 0:
                    nup, grace = renew(eps), grace0
                break
            if over:
                rec["n_over"] += 1
            rT, _ = m.move(r, v, T)
            sh = oracle.stream_block(seed, eid, oracle.SCAT_HI, k)
            sl = oracle.stream_block(seed, eid, oracle.SCAT_LO, k)
            n = _iso(oracle.uniform53(sh[0], sl[0]), oracle.uniform53(sh[1], sl[1]))
            v2 = vT[0] * vT[0] + vT[1] * vT[1] + vT[2] * vT[2]
            cos_t = (n[0] * vT[0] + n[1] * vT[1] + n[2] * vT[2]) / math.sqrt(v2)
            epsp = max(oracle.energy_after(kind, eps, thr, cos_t, mass), 0.0)
            rec["sum_eps"] += eps
            if kind == synth.IONIZATION:
                epsp *= 0.5
                rec["G"] += 1
            elif kind == synth.ATTACHMENT:
                rec["D"] += 1
            rec["sum_epsp"] += epsp
            k += 1
            r = rT
            t += T
            T = 0.0
            v = n * _speed(epsp)
            if grace == 0:
                nup, grace = renew(epsp), grace0
            break
    rec.update(k_end=k, blocks=block, r=r, t=t)
    return rec


@pytest.mark.parametrize("i,zeta,grace", [(0, 0.25, 50), (21, 0.1, 7), (31, 0.5, 300), (31, 0.05, 1),
                                          (12, 1.0, 3)])
def test_brute_force_records(i, zeta, grace):
    cfg = _variable(synth.cfg2_argon_sweep()[i], trial_zeta=zeta, trial_grace=grace)
    m = oracle.OracleModel.from_config(cfg)
    n_e, n_c, seed = 4, 250, 17
    got = m.run(n_e, n_c, seed).records
    total_fail = 0
    for e in range(n_e):
        want = brute_force_variable(m, cfg, zeta, grace, e, n_c, seed)
        g = got[got["id"] == e][0]
        for key in ("n_null", "n_fail", "n_forbidden", "n_over", "G", "D", "blocks", "k_end"):
            assert int(g[key]) == int(want[key]), (e, key, int(g[key]), want[key])
        np.testing.assert_allclose(g["r"], want["r"], rtol=1e-12, atol=1e-18)
        for key in ("t", "sum_eps", "sum_epsp"):
            assert g[key] == pytest.approx(want[key], rel=1e-12), key
        total_fail += want["n_fail"]
    assert total_fail > 0
