"""Moving targets (section "Effect of gas temperature") on the GPU, through the C ABI, against
the FP64 oracle on the same seeded inputs: per-electron records and event sequences element by
element in FP64 (centre-of-momentum thresholds and forbidden picks included), FP32-mixed
tallies within the statistical tolerance of FP64, the zero-field relaxation to (3/2) kT in
both precisions, and batches, the pooled schedule and serving epochs that change no bit."""
import math
import time

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies as oracle_tallies
from swarm_testutil import compare_events, compare_records, tally_agreement

pytestmark = pytest.mark.gpu

QE, ME, AMU = oracle.constants()
KB = oracle.boltzmann()


def _th(cfg, T=293.0):
    return cfg.scaled(thermal_targets=1, T_K=T)


def _threshold_gas(T_K):
    el = synth.maxwell_component(1.0).channels[0]
    e = np.geomspace(0.05, 1000.0, 200)
    exc = synth.Channel(synth.EXCITATION, 0.05, e, np.full(len(e), 2e-20))
    return synth.SwarmConfig([synth.Component(1.0, 1.0, [el, exc])], synth.td_to_field(0.3),
                             init_energy_eV=0.06, T_K=T_K, thermal_targets=1)


CASES = [
    ("argon-1Td", lambda: _th(synth.cfg2_argon_sweep()[0])),
    ("argon-100Td-2000K", lambda: _th(synth.cfg2_argon_sweep()[21], 2000.0)),
    ("argon-1e-3Td", lambda: _th(synth.cfg2_argon_sweep()[0].scaled(E_V_per_m=synth.td_to_field(1e-3),
                                                                     init_energy_eV=0.001))),
    ("threshold-gas-3000K", lambda: _threshold_gas(3000.0)),
    ("arco2-100Td-B", lambda: _th(synth.cfg3_mixture_real().scaled(secondaries=0))),
    ("argon-30Td-coulomb", lambda: _th(synth.cfg2_argon_sweep()[16].scaled(
        components=[c.with_scattering(1) for c in synth.cfg2_argon_sweep()[16].components]))),
    ("arco2-xi-binned", lambda: _th(synth.cfg3_mixture_real().scaled(
        secondaries=0, trial_strategy=2, trial_bins=10, trial_grace=200,
        components=[c.with_scattering(2, 0.6) for c in synth.cfg3_mixture_real().components]))),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_fp64_records_and_events(gpu, name, mk):
    sw = gpu
    cfg = mk()
    ids = list(range(6))
    n_e, n_c, seed = 400, 300, 11
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.set_trace(ids, 1024)
    s.run(n_e, n_c, seed)
    r = oracle.OracleModel.from_config(cfg).run(n_e, n_c, seed, trace_ids=ids, max_events=1024)
    compare_records(s.records(), r.records)
    ev, cnt = s.trace_events()
    compare_events(ev, cnt, r.events, ids)
    T = s.tallies()
    O = oracle_tallies(r.records)
    for key in ("n_real", "n_null", "n_forbidden", "n_fail"):
        assert T[key] == O[key], key


def test_fp64_threshold_in_cm_frame(gpu):
    """Excitations below the laboratory onset and forbidden picks above it, as in the oracle."""
    sw = gpu
    cfg = _threshold_gas(3000.0)
    ids = list(range(64))
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.set_trace(ids, 2048)
    s.run(64, 1500, 4)
    ev, cnt = s.trace_events()
    r = oracle.OracleModel.from_config(cfg).run(64, 1500, 4, trace_ids=ids, max_events=2048)
    compare_events(ev, cnt, r.events, ids)
    onset = 0.05 * (ME + AMU) / AMU
    flat = np.concatenate([ev[i, :cnt[i]] for i in range(len(ids))])
    below = (flat["type"] == 1) & (flat["channel"] == 1) & (flat["eps"] < onset)
    above = (flat["type"] == 2) & (flat["eps"] >= onset)
    assert below.any() and above.any()


def test_fp64_real_secondaries_thermal(gpu):
    sw = gpu
    cfg = _th(synth.cfg3_mixture_real(n_electrons=48, n_collisions=1200), 1000.0)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.run(48, 1200, 4)
    r = oracle.OracleModel.from_config(cfg).run(48, 1200, 4)
    g = s.records()
    assert len(g) > 48
    compare_records(g, r.records)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("eps0,T,M_amu,n", [(1.0, 293.0, 1.0, 3000), (0.001, 600.0, 4.0, 2000)])
def test_zero_field_relaxation_closed_form(gpu, precision, eps0, T, M_amu, n):
    sw = gpu
    cfg = synth.SwarmConfig([synth.maxwell_component(M_amu)], 0.0, init_energy_eV=eps0, T_K=T,
                            thermal_targets=1)
    s = sw.Swarm.from_config(cfg, precision)
    s.run(50000, n, 7)
    Tl = s.tallies()
    M = M_amu * AMU
    kappa = 2 * ME * M / (ME + M) ** 2
    eth = 1.5 * KB * T / QE
    mean = eth + (eps0 - eth) * (1 - (1 - kappa) ** n) / (n * kappa)
    v, sig, _ = Tl["mean_energy"]
    # FP32: the energy after a collision is rounded to single precision (relative 2^-24 per
    # collision, unbiased): within the statistical allowance plus 1e-5
    assert abs(v - mean) < 4 * sig + 1e-5 * mean, (v, mean, sig)


@pytest.mark.parametrize("i", [0, 12, 21])
def test_fp32_thermal_tallies_match_fp64(gpu, i):
    sw = gpu
    cfg = _th(synth.cfg2_argon_sweep()[i], 1000.0)
    t = {}
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        s = sw.Swarm.from_config(cfg, prec)
        s.run(20000, 2000, 1)
        t[prec] = s.tallies()
    bad = tally_agreement(t[sw.SWARM_FP32_MIXED], t[sw.SWARM_FP64],
                          keys=["W", "mean_energy", "mean_energy_after", "D", "DL", "DT"])
    assert not bad, bad


def test_batch_mixes_kernel_levels(gpu):
    """Targets at rest, adaptive trial frequencies and moving targets in one launch (the
    moving-target kernel serves them all): each as in its own run."""
    sw = gpu
    base = [synth.cfg2_argon_sweep()[i] for i in (3, 14, 25)]
    cfgs = base + [c.scaled(trial_strategy=1) for c in base] + [_th(c, 500.0) for c in base]
    jobs = [(3000, 700, 5 + i) for i in range(len(cfgs))]
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        hs = [sw.Swarm.from_config(c, prec) for c in cfgs]
        sw.swarm_batch_run([h.h for h in hs], jobs, {"use_graph": 1})
        for c, h, j in zip(cfgs, hs, jobs):
            s = sw.Swarm.from_config(c, prec)
            s.run(*j)
            assert h.records().tobytes() == s.records().tobytes(), (c.label, c.thermal_targets, prec)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_pooled_schedule_thermal(gpu, precision):
    sw = gpu
    sweep = synth.cfg2_argon_sweep()
    cfgs = [_th(sweep[2]), _th(sweep[17], 2000.0), _threshold_gas(3000.0),
            _th(synth.cfg3_mixture_real().scaled(secondaries=0))]
    jobs = [(1500 + 97 * i, 300 + 41 * i, 3 + i) for i in range(len(cfgs))]
    ref = [sw.Swarm.from_config(c, precision) for c in cfgs]
    sw.swarm_batch_run([h.h for h in ref], jobs, {"block_size": 128, "pending_trigger": 24})
    hs = [sw.Swarm.from_config(c, precision) for c in cfgs]
    sw.swarm_batch_run([h.h for h in hs], jobs, {"block_size": 256, "service_waves": 1, "chunk": 1024})
    for c, a, b in zip(cfgs, ref, hs):
        assert a.records().tobytes() == b.records().tobytes(), c.label


def test_server_epochs_keep_thermal_results(gpu):
    sw = gpu
    reqs = [_th(synth.cfg5_request(i).scaled(n_electrons=5000, n_collisions=900), 800.0) for i in range(4)]
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        alone = []
        for c in reqs:
            s = sw.Swarm.from_config(c, prec)
            s.run(c.n_electrons, c.n_collisions, c.seed)
            alone.append(s.tallies())
        srv = sw.swarm_server_create(32 << 30, prec, quantum_collisions=128)
        try:
            tickets = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, prec),
                                              c.n_electrons, c.n_collisions, c.seed) for c in reqs]
            t0 = time.time()
            got = {}
            while len(got) < len(tickets):
                for t in tickets:
                    if t not in got:
                        done, tal, _ = sw.swarm_server_poll(srv, t)
                        if done:
                            got[t] = tal
                assert time.time() - t0 < 120
                time.sleep(0.01)
            for t, a, c in zip(tickets, alone, reqs):
                assert got[t] == a, (prec, c.label)
        finally:
            sw.swarm_server_destroy(srv)


def test_invalid_thermal_refused(gpu):
    sw = gpu
    for T, flag in ((-1.0, 1), (float("nan"), 1), (293.0, 2)):
        with pytest.raises(sw.SwarmError):
            sw.Swarm.from_config(synth.cfg1_maxwell().scaled(T_K=T, thermal_targets=flag), sw.SWARM_FP64)
