"""The binned trial frequency (section "Trial frequency strategies", BinnedTrialFrequency) on
the GPU, through the C ABI, against the FP64 oracle on the same seeded inputs: per-electron
records and event sequences (fails and the flag of a failed retry included) element by
element in FP64, FP32-mixed tallies within the statistical tolerance of FP64, a constant-
rate gas that never fails, batches that mix all three strategies, serving epochs and the
pooled schedule that change nothing."""
import time

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies as oracle_tallies
from swarm_testutil import compare_events, compare_records, tally_agreement

pytestmark = pytest.mark.gpu

QE, ME, AMU = oracle.constants()


def _bin(cfg, bins=10, grace=5000):
    return cfg.scaled(trial_strategy=2, trial_bins=bins, trial_grace=grace)


CASES = [
    ("argon-1Td", lambda: _bin(synth.cfg2_argon_sweep()[0])),
    ("argon-1Td-b30-grace50", lambda: _bin(synth.cfg2_argon_sweep()[0], 30, 50)),
    ("argon-100Td-grace7", lambda: _bin(synth.cfg2_argon_sweep()[21], 10, 7)),
    ("argon-1000Td-b4-grace300", lambda: _bin(synth.cfg2_argon_sweep()[31], 4, 300)),
    ("argon-1000Td-b20-grace1", lambda: _bin(synth.cfg2_argon_sweep()[31], 20, 1)),
    ("arco2-100Td-B-b7-grace200", lambda: _bin(synth.cfg3_mixture_real().scaled(secondaries=0), 7, 200)),
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
    g = s.records()
    compare_records(g, r.records)
    ev, cnt = s.trace_events()
    compare_events(ev, cnt, r.events, ids)
    T = s.tallies()
    O = oracle_tallies(r.records)
    for key in ("n_real", "n_null", "n_forbidden", "n_fail"):
        assert T[key] == O[key], key
    assert abs(T["efficiency"] - O["efficiency"]) < 1e-14
    assert O["n_fail"] > 0


def test_fp64_retry_failures_flagged(gpu):
    """Many retries fail again here (flag 16); the flags agree electron by electron."""
    sw = gpu
    cfg = _bin(synth.cfg2_argon_sweep()[21], 30, 50)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.run(2000, 400, 3)
    r = oracle.OracleModel.from_config(cfg).run(2000, 400, 3)
    compare_records(s.records(), r.records)
    assert int(((r.records["flags"] & 16) != 0).sum()) > 100


@pytest.mark.parametrize("P,bins", [(16, 100), (4, 50)])
def test_fp64_coarse_grid_empty_bins(gpu, P, bins):
    """A coarse rate grid with many bins per decade leaves bins without a node (nu' 0);
    only the range maximum after a fail passes over them."""
    sw = gpu
    cfg = _bin(synth.cfg2_argon_sweep()[18], bins, 40)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64, grid_points_per_octave=P)
    s.run(600, 300, 8)
    m = oracle.OracleModel.from_config(cfg, grid_P=P)
    assert (m.bins()[1] == 0).any()
    r = m.run(600, 300, 8)
    compare_records(s.records(), r.records)
    assert int(r.records["n_fail"].sum()) > 0


def test_fp64_real_secondaries_binned(gpu):
    sw = gpu
    cfg = _bin(synth.cfg3_mixture_real(n_electrons=48, n_collisions=1200), 10, 100)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.run(48, 1200, 4)
    r = oracle.OracleModel.from_config(cfg).run(48, 1200, 4)
    g = s.records()
    assert len(g) > 48
    compare_records(g, r.records)
    assert int(r.records["n_fail"].sum()) > 0


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_constant_rate_gas_never_fails(gpu, precision):
    sw = gpu
    cfg = synth.cfg1_maxwell(n_electrons=20000, n_collisions=2000).scaled(
        user_majorant=4e12, trial_strategy=2, trial_bins=10, trial_grace=50)
    s = sw.Swarm.from_config(cfg, precision)
    s.run(cfg.n_electrons, cfg.n_collisions, 1)
    T = s.tallies()
    assert T["n_fail"] == 0
    assert T["efficiency"] > 1 - 1e-4
    W = QE * synth.td_to_field(10.0) / (ME * 1e12)
    assert abs(T["W"][0] - W) < 3.5 * T["W"][1] + 1e-3 * W


@pytest.mark.parametrize("i", [0, 10, 21, 31])
def test_fp32_binned_tallies_match_fp64(gpu, i):
    sw = gpu
    cfg = _bin(synth.cfg2_argon_sweep()[i], 10, 5000)
    t = {}
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        s = sw.Swarm.from_config(cfg, prec)
        s.run(20000, 2000, 1)
        t[prec] = s.tallies()
    bad = tally_agreement(t[sw.SWARM_FP32_MIXED], t[sw.SWARM_FP64],
                          keys=["W", "mean_energy", "mean_energy_after", "D", "DL", "DT"])
    assert not bad, bad
    a, b = t[sw.SWARM_FP32_MIXED], t[sw.SWARM_FP64]
    assert abs(a["efficiency"] / b["efficiency"] - 1) < 0.01
    assert b["n_fail"] > 0


def test_batch_mixes_all_strategies(gpu):
    """Constant, variable and binned instances in one persistent launch: each as in its own run."""
    sw = gpu
    base = [synth.cfg2_argon_sweep()[i] for i in (3, 14, 25)]
    cfgs = base + [c.scaled(trial_strategy=1) for c in base] + [_bin(c, 10, 60) for c in base]
    jobs = [(3000, 700, 5 + i) for i in range(len(cfgs))]
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        hs = [sw.Swarm.from_config(c, prec) for c in cfgs]
        sw.swarm_batch_run([h.h for h in hs], jobs, {"use_graph": 1})
        for c, h, j in zip(cfgs, hs, jobs):
            s = sw.Swarm.from_config(c, prec)
            s.run(*j)
            assert h.records().tobytes() == s.records().tobytes(), (c.label, c.trial_strategy, prec)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_pooled_schedule_binned(gpu, precision):
    sw = gpu
    sweep = synth.cfg2_argon_sweep()
    cfgs = [_bin(sweep[2], 30, 50), _bin(sweep[17], 10, 5000), _bin(sweep[30], 20, 1),
            _bin(synth.cfg3_mixture_real().scaled(secondaries=0), 7, 200)]
    jobs = [(1500 + 97 * i, 300 + 41 * i, 3 + i) for i in range(len(cfgs))]
    ref = [sw.Swarm.from_config(c, precision) for c in cfgs]
    sw.swarm_batch_run([h.h for h in ref], jobs, {"block_size": 128, "pending_trigger": 24})
    hs = [sw.Swarm.from_config(c, precision) for c in cfgs]
    sw.swarm_batch_run([h.h for h in hs], jobs, {"block_size": 256, "service_waves": 1, "chunk": 1024})
    for c, a, b in zip(cfgs, ref, hs):
        assert a.records().tobytes() == b.records().tobytes(), c.label


def test_server_epochs_keep_binned_results(gpu):
    sw = gpu
    reqs = [_bin(synth.cfg5_request(i).scaled(n_electrons=5000, n_collisions=900), 10, 300) for i in range(4)]
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


def test_invalid_binned_refused(gpu):
    sw = gpu
    for bins, grace in ((101, 10), (-1, 10), (10, -3)):
        with pytest.raises(sw.SwarmError):
            sw.Swarm.from_config(_bin(synth.cfg2_argon_sweep()[3], bins, grace), sw.SWARM_FP64)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_tallies_flag_inexact_strategies_and_count_failed_retries(gpu, precision):
    """The tallies say whether the run used the exact constant trial frequency, and count the
    electrons whose binned retry failed again (record flag 16)."""
    sw = gpu
    base = synth.cfg2_argon_sweep()[12]
    for cfg, strategy in ((base, 0), (base.scaled(trial_strategy=1), 1), (_bin(base, 10, 50), 2)):
        s = sw.Swarm.from_config(cfg, precision)
        s.run(4000, 800, 6)
        T = s.tallies()
        assert T["trial_strategy"] == strategy
        assert T["exact"] == (1 if strategy == 0 else 0)
        n16 = int(((s.records()["flags"] & 16) != 0).sum())
        assert T["n_retry_failed"] == n16
        if strategy == 2:
            assert n16 > 0
