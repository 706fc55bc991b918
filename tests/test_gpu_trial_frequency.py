"""The variable trial frequency (section "Trial frequency strategies") on the GPU, through
the C ABI, against the FP64 oracle on the same seeded inputs: per-electron records and
event sequences (fails included) element by element in FP64, FP32-mixed tallies within the
statistical tolerance of FP64, the capped strategy equal to the constant one, mixed
strategies in one batch, and a serving epoch split that changes nothing."""
import time

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies as oracle_tallies
from swarm_testutil import compare_events, compare_records, tally_agreement

pytestmark = pytest.mark.gpu


def _var(cfg, **kw):
    return cfg.scaled(trial_strategy=1, **kw)


CASES = [
    ("argon-1Td", lambda: _var(synth.cfg2_argon_sweep()[0])),
    ("argon-100Td", lambda: _var(synth.cfg2_argon_sweep()[21])),
    ("argon-1000Td-grace50", lambda: _var(synth.cfg2_argon_sweep()[31], trial_grace=50)),
    ("arco2-100Td-B-zeta0.1", lambda: _var(synth.cfg3_mixture_real().scaled(secondaries=0), trial_zeta=0.1,
                                          trial_grace=200)),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_fp64_records_and_events_with_fails(gpu, name, mk):
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


def test_fp64_real_secondaries_variable(gpu):
    sw = gpu
    cfg = _var(synth.cfg3_mixture_real(n_electrons=48, n_collisions=1200), trial_grace=100)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.run(48, 1200, 4)
    r = oracle.OracleModel.from_config(cfg).run(48, 1200, 4)
    g = s.records()
    assert len(g) > 48
    compare_records(g, r.records)
    assert int(r.records["n_fail"].sum()) > 0


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_capped_variable_equals_constant(gpu, precision):
    sw = gpu
    cfg = synth.cfg2_argon_sweep()[12]
    a = sw.Swarm.from_config(cfg, precision)
    a.run(2000, 400, 8)
    b = sw.Swarm.from_config(_var(cfg, trial_zeta=1e30, trial_grace=3), precision)
    b.run(2000, 400, 8)
    ra, rb = a.records(), b.records()
    assert ra.tobytes() == rb.tobytes()


@pytest.mark.parametrize("i", [0, 10, 21, 31])
def test_fp32_variable_tallies_match_fp64(gpu, i):
    sw = gpu
    cfg = _var(synth.cfg2_argon_sweep()[i])
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


def test_batch_mixes_strategies(gpu):
    """Constant and variable instances in one persistent launch: each as in its own run."""
    sw = gpu
    cfgs = [synth.cfg2_argon_sweep()[i] for i in (3, 14, 25)]
    cfgs = cfgs + [_var(c) for c in cfgs]
    jobs = [(3000, 700, 5 + i) for i in range(len(cfgs))]
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        hs = [sw.Swarm.from_config(c, prec) for c in cfgs]
        sw.swarm_batch_run([h.h for h in hs], jobs, {"use_graph": 1})
        for c, h, j in zip(cfgs, hs, jobs):
            s = sw.Swarm.from_config(c, prec)
            s.run(*j)
            assert h.records().tobytes() == s.records().tobytes(), (c.label, c.trial_strategy, prec)


def test_server_epochs_keep_variable_results(gpu):
    """Serving splits a request into epochs at real-collision boundaries; the trial
    frequency and its grace count carry over, so the bits do not change."""
    sw = gpu
    reqs = [_var(synth.cfg5_request(i).scaled(n_electrons=5000, n_collisions=900), trial_grace=300)
            for i in range(4)]
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
