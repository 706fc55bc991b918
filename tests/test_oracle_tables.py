"""Pins of the table extension (section 'Extension of the cross-section tables'), the rate
tables of eq. (frequency) on the octave grid, the interpolation and the channel selection."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth.tables import Channel, Component, ELASTIC, EXCITATION, IONIZATION, ATTACHMENT

QE, ME, AMU = oracle.constants()


def _one(channels, mass=40.0, E=1e5, N=2.5e25):
    return oracle.OracleModel([Component(mass, 1.0, channels)], E, N_per_m3=N)


def _elastic_powerlaw(A=3e-20, K=-0.7):
    e = np.geomspace(0.05, 100.0, 40)
    return Channel(ELASTIC, 0.0, e, A * e ** K), A, K


def test_right_extension_reproduces_power_law():
    ch, A, K = _elastic_powerlaw()
    m = _one([ch])
    for eps in (150.0, 400.0, 2000.0, 1e4):
        assert abs(m.sigma_raw(0, eps) / (A * eps ** K) - 1) < 1e-12


def test_left_extension_elastic_is_constant():
    ch, A, K = _elastic_powerlaw()
    m = _one([ch])
    for eps in (1e-5, 1e-3, 0.05):
        assert m.sigma_raw(0, eps) == ch.sigma_m2[0]


def test_inelastic_zero_below_threshold_and_ramp_from_threshold():
    el, _, _ = _elastic_powerlaw()
    e = np.array([12.0, 20.0, 50.0])
    s = np.array([1e-21, 3e-21, 2e-21])
    m = _one([el, Channel(EXCITATION, 10.0, e, s)])
    assert m.sigma_raw(1, 9.999) == 0.0
    assert m.sigma_raw(1, 10.0) == 0.0
    assert abs(m.sigma_raw(1, 11.0) - 0.5e-21) < 1e-33          # (10,0) -> (12,1e-21)
    assert abs(m.sigma_raw(1, 16.0) - 2e-21) < 1e-33            # midpoint of (12,1e-21),(20,3e-21)


def test_right_extension_zero_if_last_point_zero():
    el, _, _ = _elastic_powerlaw()
    m = _one([el, Channel(ATTACHMENT, 0.0, np.array([1.0, 2.0, 3.0]), np.array([1e-22, 1e-22, 0.0]))])
    assert m.sigma_raw(1, 10.0) == 0.0


def test_maxwell_rate_is_constant_on_grid():
    m = oracle.OracleModel([synth.maxwell_component(4.0)], 2.5e5)
    nodes, C = m.tables()
    assert C.shape == (1, 1665)
    np.testing.assert_allclose(C[0], 1e12, rtol=2e-6)
    rng = np.random.default_rng(5)
    for eps in 10 ** rng.uniform(-5, 4, 200):
        assert abs(m.nu_grid(eps)[0] / 1e12 - 1) < 2e-6


def test_grid_nodes_and_exact_node_values():
    m = oracle.OracleModel([synth.argon_like()], 1e5)
    nodes, C = m.tables()
    G = m.grid_size
    assert G == 26 * 64 + 1
    assert nodes[0] == 2.0 ** -14 and nodes[-1] == 2.0 ** 12
    assert nodes[64] == 2.0 ** -13 and nodes[65] == 2.0 ** -13 * (1 + 1 / 64)
    for g in (0, 1, 63, 64, 700, 1500, G - 2):
        v, over = m.nu_grid(nodes[g])
        assert v == C[-1, g] and not over
    v, over = m.nu_grid(nodes[-1])
    assert v == C[-1, -1] and over
    assert m.nu_grid(1e-9)[0] == C[-1, 0]
    # node values are the raw rates of eq. (frequency): n sigma sqrt(2 eps/m)
    for g in (100, 900, 1400):
        assert abs(C[-1, g] / m.rate_raw_total(nodes[g]) - 1) < 1e-14


def test_grid_interpolation_error_is_small():
    # resampling on 64 points per octave keeps the total rate within 0.1 % of the
    # per-collision interpolation of the raw tables (away from threshold kinks)
    for comps in ([synth.argon_like()], synth.configs.mixture_ar_co2()):
        m = oracle.OracleModel(comps, 1e5)
        rng = np.random.default_rng(6)
        worst = 0.0
        for eps in 10 ** rng.uniform(-1.9, 3, 3000):
            g = m.nu_grid(eps)[0]
            r = m.rate_raw_total(eps)
            worst = max(worst, abs(g / r - 1))
        assert worst < 2e-2
        errs = [abs(m.nu_grid(e)[0] / m.rate_raw_total(e) - 1) for e in 10 ** rng.uniform(-1.9, 3, 3000)]
        assert np.median(errs) < 1e-3


def test_majorant_is_lazy_maximum():
    m = oracle.OracleModel(synth.configs.mixture_ar_co2(), 1e5)
    nodes, C = m.tables()
    assert m.majorant == (1 + 2.0 ** -20) * C[-1].max()
    assert np.all(np.diff(C, axis=0) >= 0)    # cumulative over channels


def test_fixed_majorant_below_maximum_is_refused():
    comps = [synth.argon_like()]
    m = oracle.OracleModel(comps, 1e5)
    with pytest.raises(ValueError):
        oracle.OracleModel(comps, 1e5, user_majorant=0.5 * m.majorant)
    m2 = oracle.OracleModel(comps, 1e5, user_majorant=2 * m.majorant)
    assert m2.majorant == 2 * m.majorant


@pytest.mark.parametrize("bad", ["order", "negative", "fraction", "nan"])
def test_invalid_tables_are_refused(bad):
    e = np.array([1.0, 2.0, 3.0])
    s = np.array([1e-20, 2e-20, 1e-20])
    frac = 1.0
    if bad == "order":
        e = np.array([1.0, 3.0, 2.0])
    elif bad == "negative":
        s = np.array([1e-20, -1e-21, 1e-20])
    elif bad == "fraction":
        frac = 0.9
    elif bad == "nan":
        s = np.array([1e-20, np.nan, 1e-20])
    with pytest.raises(ValueError):
        oracle.OracleModel([Component(4.0, frac, [Channel(ELASTIC, 0.0, e, s)])], 1e5)


def test_channel_selection_frequencies():
    # at a fixed energy, x = R nu' uniform on [0, nu') selects channel c with probability
    # nu_c(eps)/nu' and gives a null collision with probability 1 - nu(eps)/nu'
    m = oracle.OracleModel(synth.configs.mixture_ar_co2(), 1e5)
    nc = m.n_channels
    for eps in (0.3, 5.0, 14.5, 60.0):
        cum = np.array([m.channel_cum(c, eps) for c in range(nc)])
        rates = np.diff(np.concatenate([[0.0], cum]))
        n = 200000
        xs = (np.arange(n) + 0.5) / n * m.majorant
        sel = np.array([m.select(eps, x) for x in xs])
        frac_null = np.mean(sel < 0)
        assert abs(frac_null - (1 - cum[-1] / m.majorant)) < 2.0 / n
        counts = np.bincount(sel[sel >= 0], minlength=nc) / n
        np.testing.assert_allclose(counts, rates / m.majorant, atol=2.0 / n)
