"""Anisotropic scattering (section "Theoretical framework": screened Coulomb for atoms, the
xi form for molecules) on the GPU, through the C ABI, against the FP64 oracle: records and
event sequences element by element in FP64, FP32 tallies within the statistical tolerance,
the Maxwell-gas drift eE/(m nu (1 - <cos>)) and batches that mix the models."""
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


def _with(cfg, models):
    comps = [c.with_scattering(*m) for c, m in zip(cfg.components, models)]
    return cfg.scaled(components=comps)


def _mixture_b():
    cfg = synth.cfg3_mixture_real().scaled(secondaries=0)
    return _with(cfg, [(1,), (2, 0.6)])


CASES = [
    ("argon-100Td-coulomb", lambda: _with(synth.cfg2_argon_sweep()[21], [(1,)])),
    ("argon-1000Td-coulomb", lambda: _with(synth.cfg2_argon_sweep()[31], [(1,)])),
    ("arco2-100Td-B-coulomb-xi", _mixture_b),
    ("maxwell-xi0.3", lambda: _with(synth.cfg1_maxwell(), [(2, 0.3)])),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_fp64_records_and_events(gpu, name, mk):
    sw = gpu
    cfg = mk()
    ids = list(range(6))
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.set_trace(ids, 256)
    s.run(300, 150, 21)
    r = oracle.OracleModel.from_config(cfg).run(300, 150, 21, trace_ids=ids, max_events=256)
    compare_records(s.records(), r.records)
    ev, cnt = s.trace_events()
    compare_events(ev, cnt, r.events, ids)


@pytest.mark.parametrize("n_c,rtol", [(400, 1e-9), (800, 1e-6)])
def test_fp64_real_secondaries_anisotropic(gpu, n_c, rtol):
    # Every decision (integer fields) is identical.  With anisotropic scattering the new
    # direction is a rotation of the incoming one, so the last-bit differences of the
    # device and host sin/cos carry over from collision to collision instead of being reset
    # by a fresh isotropic direction; continuous values drift apart slowly along a lineage
    # (800 collisions: lineages of ~900 electrons, within the default capacity).
    sw = gpu
    cfg = _with(synth.cfg3_mixture_real(n_electrons=40, n_collisions=n_c), [(1,), (2, 0.5)])
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.run(40, n_c, 9)
    r = oracle.OracleModel.from_config(cfg).run(40, n_c, 9)
    g = s.records()
    assert len(g) > 40
    compare_records(g, r.records, rtol=rtol)


@pytest.mark.parametrize("name,mk", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_fp32_tallies_match_fp64(gpu, name, mk):
    sw = gpu
    cfg = mk()
    t = {}
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        s = sw.Swarm.from_config(cfg, prec)
        s.run(20000, 1500, 2)
        t[prec] = s.tallies()
    bad = tally_agreement(t[sw.SWARM_FP32_MIXED], t[sw.SWARM_FP64],
                          keys=["W", "Wx", "Wy", "mean_energy", "mean_energy_after", "D", "DL", "DT"])
    assert not bad, bad


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_maxwell_drift_closed_form(gpu, precision):
    sw = gpu
    r = 0.4
    cfg = _with(synth.cfg1_maxwell(), [(2, r)])
    s = sw.Swarm.from_config(cfg, precision)
    s.run(30000, 6000, 5)
    T = s.tallies()
    W = QE * synth.td_to_field(10.0) / (ME * 1e12 * r)
    assert abs(T["W"][0] - W) < 3.5 * T["W"][1] + 2e-3 * W, (T["W"], W)


def test_batch_mixes_scattering_models(gpu):
    sw = gpu
    base = synth.cfg2_argon_sweep()
    cfgs = [base[4], _with(base[4], [(1,)]), _with(base[18], [(2, 0.7)]), _mixture_b(), base[27]]
    jobs = [(2500, 500, 11 + i) for i in range(len(cfgs))]
    for prec in (sw.SWARM_FP64, sw.SWARM_FP32_MIXED):
        hs = [sw.Swarm.from_config(c, prec) for c in cfgs]
        sw.swarm_batch_run([h.h for h in hs], jobs, {"use_graph": 1})
        for c, h, j in zip(cfgs, hs, jobs):
            s = sw.Swarm.from_config(c, prec)
            s.run(*j)
            assert h.records().tobytes() == s.records().tobytes()


def test_invalid_scattering_refused(gpu):
    sw = gpu
    cfg = _with(synth.cfg1_maxwell(), [(2, 1.5)])
    with pytest.raises(sw.SwarmError):
        sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    cfg = _with(synth.cfg1_maxwell(), [(3,)])
    with pytest.raises(sw.SwarmError):
        sw.Swarm.from_config(cfg, sw.SWARM_FP64)


def test_server_keeps_scattering_model(gpu):
    """Served requests keep their components' scattering models: each equals its own run."""
    sw = gpu
    models = [[(1,)], [(2, 0.4)], [(0,)], [(1,)]]
    reqs = []
    for i, mdl in enumerate(models):
        c = synth.cfg5_request(i).scaled(n_electrons=3000, n_collisions=600)
        comps = [comp.with_scattering(*mdl[0]) for comp in c.components]
        reqs.append(c.scaled(components=comps))
    srv = sw.swarm_server_create(32 << 30, sw.SWARM_FP32_MIXED, quantum_collisions=200)
    try:
        tickets = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons,
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
    for t, c in zip(tickets, reqs):
        s = sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED)
        s.run(c.n_electrons, c.n_collisions, c.seed)
        assert got[t] == s.tallies(), c.label
