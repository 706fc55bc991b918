"""Serving: requests admitted by HBM budget and advanced together in epochs give the same
bits as the same request run alone, under either schedule (every admitted request in every
epoch, or shortest remaining work first)."""
import time

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies as oracle_tallies
from swarm_testutil import compare_records

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


@pytest.mark.parametrize("schedule", [0, 1], ids=["all", "shortest-first"])
def test_per_request_quanta_give_the_single_run_bits(gpu, schedule):
    """Quanta sized per request (quantum_collisions = 0: fewer real collisions per epoch for a
    gas that draws more null trials per real collision, once that has been measured): requests
    of the argon-like sweep from 1 to 1000 Td, served together over several epochs, give the
    bits of their single runs."""
    sw = gpu
    sweep = synth.cfg2_argon_sweep(n_electrons=100_000, n_collisions=20_000)
    reqs = [sweep[i] for i in (0, 10, 21, 31)]
    alone = _alone(sw, reqs, sw.SWARM_FP32_MIXED)
    srv = sw.swarm_server_create(64 << 30, sw.SWARM_FP32_MIXED, quantum_collisions=0, schedule=schedule)
    try:
        tickets = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons,
                                          c.n_collisions, c.seed) for c in reqs]
        res = _wait_all(sw, srv, tickets)
        for t, a in zip(tickets, alone):
            assert res[t][0] == a
        assert max(res[t][1]["epochs"] for t in tickets) >= 3
    finally:
        sw.swarm_server_destroy(srv)


def test_measured_blocks_per_real_match_the_records(gpu):
    """The server measures a request's trial blocks per real collision by a reduction over its
    electrons' state after the request's first epoch: for requests that finish in that epoch it
    is the records' block counts summed over the request's real collisions."""
    sw = gpu
    reqs = [_shrink(c, 20000, 800) for c in _requests(4)]
    srv = sw.swarm_server_create(64 << 30, sw.SWARM_FP32_MIXED, quantum_collisions=1000)
    recs = {}
    try:
        tickets = []
        for c in reqs:
            t, rec = sw.swarm_server_submit_records(srv, c.components, sw.params_from_config(c, 1), c.n_electrons,
                                                    c.n_collisions, c.seed)
            tickets.append(t)
            recs[t] = rec
        res = _wait_all(sw, srv, tickets)
    finally:
        sw.swarm_server_destroy(srv)
    for t in tickets:
        tal, info = res[t]
        assert info["epochs"] == 1
        blocks = float(recs[t]["blocks"].astype(np.float64).sum())
        assert blocks >= tal["n_real"]       # a block serves at most one real collision
        assert info["blocks_per_real"] == pytest.approx(blocks / tal["n_real"], rel=1e-12)


def _alone(sw, reqs, precision):
    out = []
    for c in reqs:
        s = sw.Swarm.from_config(c, precision)
        s.run(c.n_electrons, c.n_collisions, c.seed)
        out.append(s.tallies())
    return out


def test_budget_admission_queues_requests(gpu):
    sw = gpu
    reqs = [_shrink(c, 50000, 500) for c in _requests(6)]
    alone = _alone(sw, reqs, sw.SWARM_FP32_MIXED)
    srv = sw.swarm_server_create(30 << 20, sw.SWARM_FP32_MIXED, quantum_collisions=0)
    try:
        tickets = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons,
                                          c.n_collisions, c.seed) for c in reqs]
        sw.swarm_server_drain(srv)
        res = _wait_all(sw, srv, tickets)
        admits = [res[t][1]["admit_s"] for t in tickets]
        assert admits == sorted(admits)
        # the budget held some requests back until others had finished
        assert max(admits) > min(res[t][1]["done_s"] for t in tickets)
        for t, c, a in zip(tickets, reqs, alone):
            assert res[t][0]["n_real"] == c.n_electrons * c.n_collisions
            assert res[t][0] == a
    finally:
        sw.swarm_server_destroy(srv)


def test_requests_submitted_while_epochs_run(gpu):
    """Requests that arrive while others are on the device join later epochs and still give
    the bits of their single runs."""
    sw = gpu
    reqs = [_shrink(c, 20000, 2000) for c in _requests(8)]
    alone = _alone(sw, reqs, sw.SWARM_FP32_MIXED)
    srv = sw.swarm_server_create(64 << 30, sw.SWARM_FP32_MIXED, quantum_collisions=50)
    try:
        first = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons,
                                        c.n_collisions, c.seed) for c in reqs[:3]]
        t0 = time.time()
        while sw.swarm_server_poll(srv, first[0])[2]["admit_s"] == 0.0:
            assert time.time() - t0 < 60
            time.sleep(0.001)
        late = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons,
                                       c.n_collisions, c.seed) for c in reqs[3:]]
        res = _wait_all(sw, srv, first + late)
        first_admit = res[first[0]][1]["admit_s"]
        for t in late:
            assert res[t][1]["admit_s"] > first_admit
        for t, a in zip(first + late, alone):
            assert res[t][0] == a
    finally:
        sw.swarm_server_destroy(srv)


def test_served_requests_match_the_oracle(gpu):
    """Config-5 requests (random mixtures, fields and sizes, shrunk to what the oracle runs in
    seconds), served in FP64 with small epochs: every request's tallies equal the oracle's
    (continuous values to 1e-8 relative, counts exactly) and the records of those submitted
    with a record buffer equal the oracle's (integer fields exactly, continuous to 1e-9)."""
    sw = gpu
    reqs = [_shrink(c, 300, 250) for c in _requests(12)]
    srv = sw.swarm_server_create(8 << 30, sw.SWARM_FP64, quantum_collisions=40)
    recs = {}
    try:
        tickets = []
        for i, c in enumerate(reqs):
            p = sw.params_from_config(c, sw.SWARM_FP64)
            if i % 3 == 0:
                t, rec = sw.swarm_server_submit_records(srv, c.components, p, c.n_electrons, c.n_collisions, c.seed)
                recs[t] = rec
            else:
                t = sw.swarm_server_submit(srv, c.components, p, c.n_electrons, c.n_collisions, c.seed)
            tickets.append(t)
        res = _wait_all(sw, srv, tickets)
    finally:
        sw.swarm_server_destroy(srv)
    for t, c in zip(tickets, reqs):
        r = oracle.OracleModel.from_config(c).run(c.n_electrons, c.n_collisions, c.seed)
        O = oracle_tallies(r.records)
        T = res[t][0]
        assert res[t][1]["epochs"] >= c.n_collisions // 40
        for key in ("W", "Wx", "Wy", "Wz", "mean_energy", "mean_energy_after", "D", "DL", "DT", "D_vec",
                    "DL_vec", "DT_vec", "sigma", "sigma_vec", "alpha", "eta"):
            for j in range(3):
                a, b = T[key][j], O[key][j]
                assert abs(a - b) <= 1e-8 * abs(b) + 1e-300, (c.label, key, j, a, b)
        for key in ("n_real", "n_null", "n_forbidden", "n_over", "n_electrons", "n_finished", "n_ionizations",
                    "n_attachments"):
            assert T[key] == O[key], (c.label, key)
        if t in recs:
            compare_records(recs[t], r.records)


def test_failed_epoch_fails_every_admitted_request(gpu, monkeypatch):
    """A device failure in an epoch (forced from the host: the epoch launches nothing) fails
    every admitted request, including those left out of the epoch and those admitted while it
    ran; drain returns, and the server goes on serving new requests."""
    sw = gpu
    monkeypatch.setenv("SWARM_SERVER_FAIL_EPOCH", "10")
    reqs = [_shrink(c, 3000, 3000) for c in _requests(6)]
    srv = sw.swarm_server_create(64 << 30, sw.SWARM_FP32_MIXED, quantum_collisions=20, schedule=1)
    try:
        tickets = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons,
                                          c.n_collisions, c.seed) for c in reqs]
        sw.swarm_server_drain(srv)
        failed = 0
        for t in tickets:
            try:
                # a request admitted only after the failed epoch finishes normally
                assert sw.swarm_server_poll(srv, t)[0]
            except sw.SwarmError as e:
                assert e.status == sw.SWARM_ERR_DEVICE
                failed += 1
        assert failed >= 1
        c = _shrink(_requests(7)[6], 2000, 200)
        t = sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons, c.n_collisions,
                                   c.seed)
        sw.swarm_server_drain(srv)
        assert sw.swarm_server_poll(srv, t)[0]
    finally:
        sw.swarm_server_destroy(srv)


def test_destroy_cancels_unfinished_requests(gpu):
    sw = gpu
    reqs = [synth.cfg5_request(i).scaled(n_electrons=200000, n_collisions=100000) for i in range(3)]
    srv = sw.swarm_server_create(64 << 30, sw.SWARM_FP32_MIXED)
    for c in reqs:
        sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons, c.n_collisions, c.seed)
    time.sleep(0.5)
    t0 = time.time()
    sw.swarm_server_destroy(srv)
    assert time.time() - t0 < 20


def test_invalid_schedule_refused(gpu):
    sw = gpu
    with pytest.raises(sw.SwarmError):
        sw.swarm_server_create(1 << 30, sw.SWARM_FP32_MIXED, schedule=2)
