"""The C ABI's asynchronous run (swarm_run_async / swarm_wait) and caller-owned device memory
(swarm_create_in_arena, swarm_server_create_in_arena): the same records, bit for bit, as the
synchronous, library-allocated path, and the oracle's records."""
import numpy as np
import pytest

import oracle
import synth
from swarm_testutil import compare_records, sort_by_id

pytestmark = pytest.mark.gpu


def _mixture():
    return synth.cfg3_mixture_real().scaled(secondaries=0)     # argon:CO2, 100 Td, 1 T at 45 deg


def _same_bits(a, b):
    a, b = sort_by_id(a), sort_by_id(b)
    assert len(a) == len(b)
    assert a.tobytes() == b.tobytes()


def test_async_run_equals_sync_run_and_oracle(gpu):
    sw = gpu
    cfg = _mixture()
    n_e, n_c, seed = 2000, 300, 21
    ref = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    ref.run(n_e, n_c, seed)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.run_async(n_e, n_c, seed)
    with pytest.raises(sw.SwarmError) as ei:
        s.tallies()                          # the run is in flight
    assert ei.value.status == sw.SWARM_ERR_STATE
    with pytest.raises(sw.SwarmError):
        s.run(n_e, n_c, seed)
    assert s.wait() == sw.SWARM_OK
    with pytest.raises(sw.SwarmError) as ei:
        s.wait()                             # nothing in flight any more
    assert ei.value.status == sw.SWARM_ERR_STATE
    _same_bits(s.records(), ref.records())
    assert s.tallies() == ref.tallies()
    compare_records(s.records(), oracle.OracleModel.from_config(cfg).run(n_e, n_c, seed).records)


def test_async_runs_of_two_handles_overlap(gpu):
    import torch
    sw = gpu
    a_cfg, b_cfg = synth.cfg2_argon_sweep()[10], _mixture()
    want = []
    for cfg in (a_cfg, b_cfg):
        r = sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED)
        r.run(20000, 500, 3)
        want.append(r.records())
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    hs = [sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED, stream=st) for cfg, st in zip((a_cfg, b_cfg), streams)]
    for h in hs:
        h.run_async(20000, 500, 3)
    for h, w in zip(hs, want):
        h.wait()
        _same_bits(h.records(), w)


def test_async_real_secondaries(gpu):
    sw = gpu
    cfg = synth.cfg3_mixture_real(n_electrons=64, n_collisions=1500)
    ref = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    ref.run(64, 1500, 3)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.run_async(64, 1500, 3)
    assert s.wait() == sw.SWARM_OK
    _same_bits(s.records(), ref.records())
    compare_records(s.records(), oracle.OracleModel.from_config(cfg).run(64, 1500, 3).records)
    # the capacity error comes from swarm_wait, with the tallies of what finished
    small = sw.Swarm.from_config(synth.cfg3_mixture_real(n_electrons=64, n_collisions=4000), sw.SWARM_FP64, capacity=80)
    small.run_async(64, 4000, 3)
    with pytest.raises(sw.SwarmError) as ei:
        small.wait()
    assert ei.value.status == sw.SWARM_ERR_CAPACITY
    assert small.tallies()["n_dropped"] > 0


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_swarm_in_a_torch_arena(gpu, precision):
    import torch
    sw = gpu
    cfg = _mixture()
    n_e, n_c, seed = 3000, 200, 8
    p = sw.params_from_config(cfg, precision)
    nbytes = sw.swarm_arena_bytes(cfg.components, p, n_e)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = sw.Swarm.from_config(cfg, precision, arena=(buf.data_ptr(), nbytes))
    try:
        ref = sw.Swarm.from_config(cfg, precision)
        for n in (n_e, 1000):                # a smaller second run reuses the blocks
            ref.run(n, n_c, seed)
            s.run(n, n_c, seed)
            _same_bits(s.records(), ref.records())
            assert s.tallies() == ref.tallies()
        if precision == sw.SWARM_FP64:
            compare_records(s.records(), oracle.OracleModel.from_config(cfg).run(1000, n_c, seed).records)
        # a run beyond what the arena was sized for is refused, and the handle stays usable
        with pytest.raises(sw.SwarmError) as ei:
            s.run(40 * n_e, n_c, seed)
        assert ei.value.status == sw.SWARM_ERR_OUT_OF_MEMORY
        s.run(1000, n_c, seed)
        _same_bits(s.records(), ref.records())
    finally:
        s.close()
    # too small for the tables
    with pytest.raises(sw.SwarmError) as ei:
        sw.Swarm.from_config(cfg, precision, arena=(buf.data_ptr(), 4096))
    assert ei.value.status == sw.SWARM_ERR_OUT_OF_MEMORY
    del buf


def test_real_secondaries_in_a_torch_arena(gpu):
    import torch
    sw = gpu
    cfg = synth.cfg3_mixture_real(n_electrons=64, n_collisions=1500)
    p = sw.params_from_config(cfg, sw.SWARM_FP64, capacity=20000)
    nbytes = sw.swarm_arena_bytes(cfg.components, p, 64)
    buf = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    h = sw.swarm_create_in_arena(cfg.components, p, buf.data_ptr(), nbytes)
    try:
        sw.swarm_run(h, 64, 1500, 3)
        ref = sw.Swarm.from_config(cfg, sw.SWARM_FP64, capacity=20000)
        ref.run(64, 1500, 3)
        _same_bits(sw.swarm_records(h), ref.records())
    finally:
        sw.swarm_destroy(h)
    del buf


def test_server_in_a_torch_arena(gpu):
    import torch
    sw = gpu
    reqs = [synth.cfg5_request(i).scaled(n_electrons=5000, n_collisions=400) for i in range(6)]
    alone = []
    for c in reqs:
        r = sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED)
        r.run(c.n_electrons, c.n_collisions, c.seed)
        alone.append(r.tallies())
    nbytes = 256 << 20
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    srv = sw.swarm_server_create_in_arena(buf.data_ptr(), nbytes, precision=sw.SWARM_FP32_MIXED, quantum_collisions=100)
    try:
        tickets = [sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1), c.n_electrons,
                                          c.n_collisions, c.seed) for c in reqs]
        sw.swarm_server_drain(srv)
        for t, a in zip(tickets, alone):
            done, tal, _ = sw.swarm_server_poll(srv, t)
            assert done and tal == a
    finally:
        sw.swarm_server_destroy(srv)
    del buf
