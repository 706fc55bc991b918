"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded inputs.

FP64: per-electron records and event sequences agree element by element (integer fields
exactly, continuous fields to 1e-9 relative).  FP32-mixed: every tally agrees with the
oracle within 3 combined statistical sigma plus 0.5 % (the reading of the tolerance).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies as oracle_tallies
from swarm_testutil import compare_events, compare_records, paired_bias, paired_bias_failures, tally_agreement

pytestmark = pytest.mark.gpu


def _gpu_run(sw, cfg, precision, n_e, n_c, seed, trace_ids=None, max_events=0, **kw):
    s = sw.Swarm.from_config(cfg, precision, **kw)
    if trace_ids is not None:
        s.set_trace(trace_ids, max_events)
    st = s.run(n_e, n_c, seed)
    return s, st


CASES = [
    ("maxwell", lambda: synth.cfg1_maxwell()),
    ("argon-1Td", lambda: synth.cfg2_argon_sweep()[0]),
    ("argon-31Td", lambda: synth.cfg2_argon_sweep()[15]),
    ("argon-1000Td", lambda: synth.cfg2_argon_sweep()[31]),
    ("arco2-100Td-B", lambda: synth.cfg3_mixture_real().scaled(secondaries=0)),
    ("arco2-30Td-B90", lambda: synth.SwarmConfig(synth.configs.mixture_ar_co2(), synth.td_to_field(30.0),
                                                 B_T=2.0, B_angle_rad=math.pi / 2)),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_tables_match_oracle(gpu, name, mk):
    sw = gpu
    cfg = mk()
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    nodes, cum, maj = s.tables()
    m = oracle.OracleModel.from_config(cfg)
    onodes, ocum = m.tables()
    assert np.array_equal(nodes, onodes)
    np.testing.assert_allclose(cum, ocum, rtol=1e-13, atol=0)
    assert abs(maj / m.majorant - 1) < 1e-13


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_fp64_event_parity(gpu, name, mk):
    """Identical per-electron event sequences (trial block, position in block, channel,
    real/forbidden) over the first 100 real collisions, and identical final records."""
    sw = gpu
    cfg = mk()
    ids = list(range(8))
    n_e, n_c = 300, 100
    s, _ = _gpu_run(sw, cfg, sw.SWARM_FP64, n_e, n_c, 17, trace_ids=ids, max_events=256)
    m = oracle.OracleModel.from_config(cfg)
    r = m.run(n_e, n_c, 17, trace_ids=ids, max_events=256)
    compare_records(s.records(), r.records, rtol=1e-9)
    ev, cnt = s.trace_events()
    compare_events(ev, cnt, r.events, ids, rtol=1e-9)
    assert np.all(cnt >= 100)


@pytest.mark.parametrize("n_e", [1, 63, 257, 4099])
def test_fp64_ragged_sizes_and_chunks(gpu, n_e):
    """Electron counts that leave partial waves, work-groups and work items."""
    sw = gpu
    cfg = synth.cfg2_argon_sweep()[20]
    s, _ = _gpu_run(sw, cfg, sw.SWARM_FP64, n_e, 37, 5)
    r = oracle.OracleModel.from_config(cfg).run(n_e, 37, 5)
    compare_records(s.records(), r.records)


def test_fp64_tallies_match_oracle(gpu):
    sw = gpu
    cfg = synth.cfg3_mixture_real().scaled(secondaries=0)
    s, _ = _gpu_run(sw, cfg, sw.SWARM_FP64, 3000, 400, 2)
    T = s.tallies()
    O = oracle_tallies(oracle.OracleModel.from_config(cfg).run(3000, 400, 2).records)
    for key in ("W", "Wx", "Wy", "Wz", "mean_energy", "mean_energy_after", "D", "DL", "DT", "sigma",
                "sigmaL", "sigmaT", "D_vec", "DL_vec", "DT_vec", "alpha", "eta"):
        for j in range(3):
            a, b = T[key][j], O[key][j]
            assert abs(a - b) <= 1e-8 * abs(b) + 1e-300, (key, j, a, b)
    for key in ("n_real", "n_null", "n_forbidden", "n_over", "n_electrons", "n_finished", "n_ionizations",
                "n_attachments"):
        assert T[key] == O[key], key
    assert abs(T["efficiency"] - O["efficiency"]) < 1e-14


def test_fp64_real_secondaries_lineages(gpu):
    """Real secondaries: the same set of electrons (ids from the parent's stream), the same
    lineage budgets, attachments and records as the oracle."""
    sw = gpu
    cfg = synth.cfg3_mixture_real(n_electrons=64, n_collisions=1500)
    s, _ = _gpu_run(sw, cfg, sw.SWARM_FP64, 64, 1500, 3)
    r = oracle.OracleModel.from_config(cfg).run(64, 1500, 3)
    g = s.records()
    assert len(g) > 64
    compare_records(g, r.records)
    T = s.tallies()
    assert T["n_created"] == len(g) - 64 and T["n_dropped"] == 0


def test_real_capacity_error(gpu):
    sw = gpu
    cfg = synth.cfg3_mixture_real(n_electrons=64, n_collisions=4000)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64, capacity=80)
    with pytest.raises(sw.SwarmError) as ei:
        s.run(64, 4000, 3)
    assert ei.value.status == sw.SWARM_ERR_CAPACITY
    T = s.tallies()
    assert T["n_dropped"] > 0 and T["n_electrons"] == 80


def test_fp32_real_secondaries_statistics(gpu):
    sw = gpu
    cfg = synth.cfg3_mixture_real(n_electrons=2000, n_collisions=800)
    s, _ = _gpu_run(sw, cfg, sw.SWARM_FP32_MIXED, 2000, 800, 4)
    T = s.tallies()
    O = oracle_tallies(oracle.OracleModel.from_config(cfg).run(2000, 800, 4).records)
    assert not tally_agreement(T, O, keys=["W", "Wx", "Wy", "mean_energy", "D_vec", "alpha"])
    assert abs(T["n_electrons"] / O["n_electrons"] - 1) < 0.05


# systematic FP32 allowance of the paired-bias check (relative; see test_fp32_tallies_within_tolerance)
FP32_FLOOR = 3e-4

FP32_CASES = [
    ("maxwell", lambda: synth.cfg1_maxwell(), 1000, 10000),
    ("argon-1Td", lambda: synth.cfg2_argon_sweep()[0], 2000, 4000),
    ("argon-10Td", lambda: synth.cfg2_argon_sweep()[10], 2000, 4000),
    ("argon-100Td", lambda: synth.cfg2_argon_sweep()[21], 2000, 4000),
    ("argon-1000Td", lambda: synth.cfg2_argon_sweep()[31], 2000, 4000),
    ("arco2-100Td-B", lambda: synth.cfg3_mixture_real().scaled(secondaries=0), 2000, 3000),
]


@pytest.mark.parametrize("name,mk,n_e,n_c", FP32_CASES, ids=[c[0] for c in FP32_CASES])
def test_fp32_tallies_within_tolerance(gpu, name, mk, n_e, n_c):
    """FP32-mixed against the FP64 oracle on the same electrons and streams: every tally within
    the stated tolerance (3 combined sigma + 0.5%), and its FP32 bias within 4 standard errors
    of the per-electron paired differences plus 3e-4 relative, the systematic error of binary32
    rounding: about 7e-8 of the energy per collision, accumulated over the 1/(2m/M) collisions
    a gas needs to relax its energy (the Maxwell gas, M = 4 u: -2e-4 in the mean energy).  The
    paired errors are far below independent ones where the two precisions keep the same event
    sequence, and there the same check flags a 0.1% bias planted in the FP32 drift velocity."""
    sw = gpu
    cfg = mk()
    s, _ = _gpu_run(sw, cfg, sw.SWARM_FP32_MIXED, n_e, n_c, 11)
    T = s.tallies()
    ref = oracle.OracleModel.from_config(cfg).run(n_e, n_c, 11).records
    O = oracle_tallies(ref)
    bad = tally_agreement(T, O)
    assert not bad, bad
    assert abs(T["efficiency"] / O["efficiency"] - 1) < 0.01
    rec = s.records()
    pb = paired_bias(rec, ref)
    assert not paired_bias_failures(pb, floor=FP32_FLOOR), paired_bias_failures(pb, floor=FP32_FLOOR)
    bias, sig, w = pb["W"]
    if 4 * sig + FP32_FLOOR * abs(w) < 1e-3 * abs(w):
        planted = rec.copy()
        planted["r"] = planted["r"] * 1.001        # every z/t, so W, up by 0.1%
        assert [k for k, *_ in paired_bias_failures(paired_bias(planted, ref, ["W"]), floor=FP32_FLOOR)] == ["W"]


def test_fp32_bias_is_resolved_where_streams_stay_in_step(gpu):
    """Where FP32 and FP64 keep the same event sequence (the Maxwell gas; argon at 1000 Td), the
    paired error of W is small enough (4 sigma + the FP32 allowance below 0.08%) that a planted 0.1%
    bias in the FP32 W cannot pass."""
    sw = gpu
    for mk, n_e, n_c in ((lambda: synth.cfg1_maxwell(), 1000, 10000), (lambda: synth.cfg2_argon_sweep()[31], 2000, 4000)):
        cfg = mk()
        s, _ = _gpu_run(sw, cfg, sw.SWARM_FP32_MIXED, n_e, n_c, 11)
        pb = paired_bias(s.records(), oracle.OracleModel.from_config(cfg).run(n_e, n_c, 11).records, ["W"])
        bias, sig, w = pb["W"]
        assert 4 * sig + FP32_FLOOR * abs(w) < 0.8e-3 * abs(w), (cfg.label, sig / w)


def test_fp32_tracks_fp64_streams(gpu):
    """FP32 uses the truncated FP64 uniforms: its event sequence follows the FP64 one until
    a decision near a boundary flips."""
    sw = gpu
    cfg = synth.cfg2_argon_sweep()[15]
    ids = list(range(16))
    s32, _ = _gpu_run(sw, cfg, sw.SWARM_FP32_MIXED, 64, 200, 9, trace_ids=ids, max_events=64)
    s64, _ = _gpu_run(sw, cfg, sw.SWARM_FP64, 64, 200, 9, trace_ids=ids, max_events=64)
    e32, c32 = s32.trace_events()
    e64, c64 = s64.trace_events()
    same_first = 0
    for i in range(len(ids)):
        n = min(c32[i], c64[i], 10)
        if np.array_equal(e32[i, :n][["block", "sub", "channel"]], e64[i, :n][["block", "sub", "channel"]]):
            same_first += 1
    assert same_first >= 12


def test_maxwell_closed_forms_on_gpu(gpu):
    sw = gpu
    qe, me = 1.602176634e-19, 9.1093837015e-31
    W = qe * synth.td_to_field(10.0) / (me * 1e12)
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        s, _ = _gpu_run(sw, synth.cfg1_maxwell(), prec, 100000, 10000, 0)
        T = s.tallies()
        assert abs(T["W"][0] - W) <= 3.5 * T["W"][1] + 1e-4 * W, (prec, T["W"])
        assert abs(T["mean_energy"][0] - 26.448) <= 3.5 * T["mean_energy"][1] + 0.003, (prec, T["mean_energy"])
        assert abs(T["Wx"][0]) <= 3.5 * T["Wx"][1] and abs(T["Wy"][0]) <= 3.5 * T["Wy"][1]
        assert T["n_real"] == 100000 * 10000


def test_drude_drift_on_gpu(gpu):
    sw = gpu
    qe, me = 1.602176634e-19, 9.1093837015e-31
    E, B, ang = synth.td_to_field(10.0), 1.0, math.pi / 4
    comps = [synth.maxwell_component(4.0)]
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        s = sw.Swarm(comps, sw.make_params(E, B, ang, precision=prec))
        s.run(50000, 5000, 1)
        T = s.tallies()
        nu, om = 1e12, qe * B / me
        b = np.array([math.sin(ang), 0, math.cos(ang)])
        a = np.array([0, 0, -qe * E / me])
        bx = np.array([[0, -b[2], b[1]], [b[2], 0, -b[0]], [-b[1], b[0], 0]])
        Wd = np.linalg.solve(nu * np.eye(3) - om * bx, a)
        for i, k in enumerate(("Wx", "Wy", "Wz")):
            assert abs(T[k][0] - Wd[i]) <= 3.5 * T[k][1] + 2e-4 * abs(Wd[2]), (prec, k, T[k], Wd[i])


def test_invalid_arguments(gpu):
    sw = gpu
    comps = [synth.argon_like()]
    with pytest.raises(sw.SwarmError) as ei:
        sw.Swarm(comps, sw.make_params(1e5, N_per_m3=-1.0))
    assert ei.value.status == sw.SWARM_ERR_INVALID_ARG
    bad = synth.argon_like()
    bad.channels[0].energy_eV = bad.channels[0].energy_eV[::-1].copy()
    with pytest.raises(sw.SwarmError):
        sw.Swarm([bad], sw.make_params(1e5))
    s = sw.Swarm(comps, sw.make_params(1e5))
    maj = s.tables()[2]
    with pytest.raises(sw.SwarmError):
        sw.Swarm(comps, sw.make_params(1e5, user_majorant=0.5 * maj))
    with pytest.raises(sw.SwarmError):
        s.run(0, 10, 0)
    with pytest.raises(sw.SwarmError):
        s.run(10, 0, 0)
    with pytest.raises(sw.SwarmError) as ei:
        sw.swarm_tallies(sw.Swarm(comps, sw.make_params(1e5)).h)
    assert ei.value.status == sw.SWARM_ERR_STATE


def test_edge_no_field_and_single_collision(gpu):
    sw = gpu
    cfg = synth.cfg2_argon_sweep()[0].scaled(E_V_per_m=0.0)
    s, _ = _gpu_run(sw, cfg, sw.SWARM_FP64, 100, 1, 4)
    r = oracle.OracleModel.from_config(cfg).run(100, 1, 4)
    compare_records(s.records(), r.records)
    s, _ = _gpu_run(sw, cfg, sw.SWARM_FP64, 100, 50, 4)
    r = oracle.OracleModel.from_config(cfg).run(100, 50, 4)
    compare_records(s.records(), r.records)


def test_fixed_trial_frequency_doubles_nulls(gpu):
    sw = gpu
    cfg = synth.cfg2_argon_sweep()[10]
    s1 = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    maj = s1.tables()[2]
    s2, _ = _gpu_run(sw, cfg, sw.SWARM_FP64, 200, 300, 8, user_majorant=2 * maj)
    r = oracle.OracleModel.from_config(cfg, user_majorant=2 * maj).run(200, 300, 8)
    compare_records(s2.records(), r.records)


def test_many_channel_mixture(gpu):
    """The largest request shape: 6 components with up to 25 channels each."""
    sw = gpu
    rng = np.random.default_rng(123)
    comps = [synth.random_component(rng, fraction=1 / 6, max_inelastic=24) for _ in range(6)]
    cfg = synth.SwarmConfig(comps, synth.td_to_field(200.0), B_T=1.5, B_angle_rad=1.0)
    s, _ = _gpu_run(sw, cfg, sw.SWARM_FP64, 200, 200, 6)
    r = oracle.OracleModel.from_config(cfg).run(200, 200, 6)
    compare_records(s.records(), r.records)
