"""Serving: requests admitted by HBM budget and advanced together in epochs give the same
bits as the same request run alone, under either schedule (every admitted request in every
epoch, or shortest remaining work first)."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _requests(n):
    return [synth.cfg5_request(i) for i in range(n)]


def _shrink(cfg, cap_e=20000, cap_c=3000):
    return cfg.scaled(n_electrons=min(cfg.n_electrons, cap_e), n_collisions=min(cfg.n_collisions, cap_c))


def _wait_all(sw, srv, tickets, timeout=120):
    t0 = time.time()
    out = {}
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            done, tal, info = sw.swarm_server_poll(srv, t)
            if done:
                out[t] = (tal, info)
        assert time.time() - t0 < timeout
        time.sleep(0.01)
    return out


@pytest.mark.parametrize("schedule", [0, 1], ids=["all", "shortest-first"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_alone_equals_in_the_mix(gpu, precision, schedule):
    sw = gpu
    reqs = [_shrink(c) for c in _requests(8)]
    # alone: each request through its own single run
    alone = []
    for c in reqs:
        s = sw.Swarm.from_config(c, precision)
        s.run(c.n_electrons, c.n_collisions, c.seed)
        alone.append(s.tallies())
    # in the mix: all submitted together to a server with small epochs
    srv = sw.swarm_server_create(64 << 30, precision, quantum_collisions=300, schedule=schedule)
    try:
        tickets = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, precision),
                                          c.n_electrons, c.n_collisions, c.seed) for c in reqs]
        res = _wait_all(sw, srv, tickets)
        for t, a in zip(tickets, alone):
            tal, info = res[t]
            assert tal == a
            assert info["done_s"] >= info["admit_s"] >= info["submit_s"]
    finally:
        sw.swarm_server_destroy(srv)


def test_budget_admission_queues_requests(gpu):
    sw = gpu
    reqs = [_shrink(c, 50000, 500) for c in _requests(6)]
    srv = sw.swarm_server_create(30 << 20, sw.SWARM_FP32_MIXED, quantum_collisions=0)
    try:
        tickets = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons,
                                          c.n_collisions, c.seed) for c in reqs]
        sw.swarm_server_drain(srv)
        res = _wait_all(sw, srv, tickets)
        admits = [res[t][1]["admit_s"] for t in tickets]
        assert admits == sorted(admits)
        for t, c in zip(tickets, reqs):
            assert res[t][0]["n_real"] == c.n_electrons * c.n_collisions
    finally:
        sw.swarm_server_destroy(srv)


def test_invalid_schedule_refused(gpu):
    sw = gpu
    with pytest.raises(sw.SwarmError):
        sw.swarm_server_create(1 << 30, sw.SWARM_FP32_MIXED, schedule=2)
