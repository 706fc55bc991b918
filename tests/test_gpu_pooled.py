"""The pooled schedule (service waves serve the candidates of the trial waves of their
work-group at full width) changes only the order of work, so its records must equal,
bit for bit, those of the per-wave schedule, and through it the oracle."""
import math
import time

import numpy as np
import pytest

import oracle
import synth
from swarm_testutil import compare_records

pytestmark = pytest.mark.gpu


def _configs():
    sweep = synth.cfg2_argon_sweep()
    mix = synth.cfg3_mixture_real().scaled(secondaries=0)
    cfgs = [sweep[2], sweep[17], sweep[30], mix,
            synth.SwarmConfig(synth.configs.mixture_ar_co2(), synth.td_to_field(30.0), B_T=2.0,
                              B_angle_rad=math.pi / 2)]
    return cfgs + [c.scaled(trial_strategy=1, trial_grace=400) for c in cfgs]


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(256, 1), (512, 2), (192, 1)], ids=["3+1", "6+2", "2+1"])
def test_pooled_equals_per_wave(gpu, precision, shape):
    sw = gpu
    cfgs = _configs()
    jobs = [(1500 + 97 * i, 300 + 41 * i, 3 + i) for i in range(len(cfgs))]
    ref = [sw.Swarm.from_config(c, precision) for c in cfgs]
    sw.swarm_batch_run([h.h for h in ref], jobs, {"block_size": 128, "pending_trigger": 24})
    hs = [sw.Swarm.from_config(c, precision) for c in cfgs]
    bs, svc = shape
    sw.swarm_batch_run([h.h for h in hs], jobs, {"block_size": bs, "service_waves": svc, "chunk": bs * 4,
                                                 "use_graph": 1})
    for c, a, b in zip(cfgs, ref, hs):
        ra, rb = a.records(), b.records()
        assert len(ra) == len(rb)
        assert ra.tobytes() == rb.tobytes(), (c.label, c.trial_strategy, c.B_T)
        assert a.tallies() == b.tallies()


def test_pooled_matches_oracle_fp64(gpu):
    sw = gpu
    cfg = synth.cfg2_argon_sweep()[9]
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    sw.swarm_batch_run([s.h], [(777, 420, 6)], {"block_size": 256, "service_waves": 1})
    compare_records(s.records(), oracle.OracleModel.from_config(cfg).run(777, 420, 6).records)


def test_pooled_server_epochs(gpu):
    """Serving with the pooled schedule: each request equals its own single run."""
    sw = gpu
    reqs = [synth.cfg5_request(i).scaled(n_electrons=4000, n_collisions=700) for i in range(4)]
    alone = []
    for c in reqs:
        s = sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED)
        s.run(c.n_electrons, c.n_collisions, c.seed)
        alone.append(s.tallies())
    srv = sw.swarm_server_create(32 << 30, sw.SWARM_FP32_MIXED, quantum_collisions=150,
                                 opts={"block_size": 256, "service_waves": 1})
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
        for t, a in zip(tickets, alone):
            assert got[t] == a
    finally:
        sw.swarm_server_destroy(srv)


def test_service_waves_are_clamped(gpu):
    """Asking for as many service waves as the block has waves leaves one trial wave."""
    sw = gpu
    cfg = synth.cfg2_argon_sweep()[5]
    a = sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED)
    sw.swarm_batch_run([a.h], [(900, 200, 1)], {"block_size": 128})
    b = sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED)
    sw.swarm_batch_run([b.h], [(900, 200, 1)], {"block_size": 128, "service_waves": 5})
    assert a.records().tobytes() == b.records().tobytes()
