"""The relativistic mover (UniformFieldRelativisticChin, uniform E and B) on the GPU, through
the C ABI, against the FP64 oracle on the same seeded inputs: per-electron records and event
sequences element by element, from swarm energies to MeV electrons on a grid up to 2^24 eV,
in crossed and oblique magnetic fields (the |E| = c|B| degenerate case included), with the
binned trial frequency and real secondaries; batches that mix kernel levels, the pooled
schedule and serving epochs that change no bit; and the refused combinations."""
import time

import numpy as np
import pytest

import oracle
import synth
from swarm_testutil import compare_events, compare_records

pytestmark = pytest.mark.gpu

C = oracle.light_speed()


def _rel(cfg):
    return cfg.scaled(relativistic=1)


def _fast():
    comp = synth.maxwell_component(4.0, k=synth.tables.MAXWELL_K * 1e-3, min_exp2=-14, max_exp2=24)
    return synth.SwarmConfig([comp], 3e7, init_energy_eV=1.0, relativistic=1)


GRID24 = dict(grid_min_exp2=-14, grid_max_exp2=24)

CASES = [
    ("maxwell-10Td", lambda: _rel(synth.cfg1_maxwell()), {}),
    ("argon-1Td", lambda: _rel(synth.cfg2_argon_sweep()[0]), {}),
    ("argon-1000Td", lambda: _rel(synth.cfg2_argon_sweep()[31]), {}),
    ("argon-100Td-binned", lambda: _rel(synth.cfg2_argon_sweep()[21]).scaled(trial_strategy=2, trial_grace=50), {}),
    ("fast-keV-MeV", _fast, GRID24),
    ("maxwell-10Td-B2T-45deg", lambda: _rel(synth.cfg1_maxwell().scaled(B_T=2.0, B_angle_rad=0.785)), {}),
    ("argon-100Td-B1T-crossed", lambda: _rel(synth.cfg2_argon_sweep()[21].scaled(B_T=1.0, B_angle_rad=1.5707963267948966)), {}),
    ("fast-crossed-E=cB", lambda: _fast().scaled(B_T=0.1, B_angle_rad=1.5707963267948966), GRID24),
    ("fast-oblique", lambda: _fast().scaled(B_T=0.05, B_angle_rad=0.4), GRID24),
]


@pytest.mark.parametrize("name,mk,grid", CASES, ids=[c[0] for c in CASES])
def test_fp64_records_and_events(gpu, name, mk, grid):
    sw = gpu
    cfg = mk()
    ids = list(range(6))
    n_e, n_c, seed = 300, 300, 11
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64, **grid)
    s.set_trace(ids, 1024)
    s.run(n_e, n_c, seed)
    kw = {"grid_emax": grid["grid_max_exp2"]} if grid else {}
    r = oracle.OracleModel.from_config(cfg, **kw).run(n_e, n_c, seed, trace_ids=ids, max_events=1024)
    g = s.records()
    compare_records(g, r.records)
    ev, cnt = s.trace_events()
    compare_events(ev, cnt, r.events, ids)
    if grid:
        assert np.all(np.linalg.norm(g["r"], axis=1) / g["t"] < C)
        assert np.max(g["sum_eps"] / n_c) > 1e4


def test_fp64_real_secondaries_relativistic(gpu):
    sw = gpu
    cfg = _rel(synth.cfg3_mixture_real(n_electrons=48, n_collisions=1200))
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.run(48, 1200, 4)
    r = oracle.OracleModel.from_config(cfg).run(48, 1200, 4)
    g = s.records()
    assert len(g) > 48
    compare_records(g, r.records)


def test_refused_combinations(gpu):
    sw = gpu
    cfg = _rel(synth.cfg1_maxwell())
    with pytest.raises(sw.SwarmError):
        sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED)
    with pytest.raises(sw.SwarmError):
        sw.Swarm.from_config(cfg.scaled(thermal_targets=1), sw.SWARM_FP64)
    with pytest.raises(sw.SwarmError):
        sw.Swarm.from_config(cfg.scaled(relativistic=2), sw.SWARM_FP64)


def test_batch_and_pooled_keep_relativistic_results(gpu):
    sw = gpu
    base = [synth.cfg2_argon_sweep()[i] for i in (3, 14, 25)]
    cfgs = base + [_rel(c) for c in base] + [base[1].scaled(trial_strategy=1)]
    jobs = [(2500, 500, 5 + i) for i in range(len(cfgs))]
    alone = []
    for c, j in zip(cfgs, jobs):
        s = sw.Swarm.from_config(c, sw.SWARM_FP64)
        s.run(*j)
        alone.append(s.records())
    for opts in ({"use_graph": 1}, {"block_size": 256, "service_waves": 1, "chunk": 1024}):
        hs = [sw.Swarm.from_config(c, sw.SWARM_FP64) for c in cfgs]
        sw.swarm_batch_run([h.h for h in hs], jobs, opts)
        for c, h, a in zip(cfgs, hs, alone):
            assert h.records().tobytes() == a.tobytes(), (c.label, c.relativistic, opts)


def test_server_epochs_keep_relativistic_results(gpu):
    sw = gpu
    reqs = [_rel(synth.cfg5_request(i).scaled(n_electrons=3000, n_collisions=700)) for i in range(3)]
    alone = []
    for c in reqs:
        s = sw.Swarm.from_config(c, sw.SWARM_FP64)
        s.run(c.n_electrons, c.n_collisions, c.seed)
        alone.append(s.tallies())
    srv = sw.swarm_server_create(32 << 30, sw.SWARM_FP64, quantum_collisions=128)
    try:
        tickets = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 0), c.n_electrons,
                                          c.n_collisions, c.seed) for c in reqs]
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
    finally:
        sw.swarm_server_destroy(srv)
    for t, a, c in zip(tickets, alone, reqs):
        assert got[t] == a, c.label
