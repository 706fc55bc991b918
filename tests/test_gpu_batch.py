"""Batched persistent launches: every instance's results are bit-identical to its own
single run, for any launch shape, with and without the hipGraph, and on replays."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies as oracle_tallies
from swarm_testutil import compare_records, tally_agreement

pytestmark = pytest.mark.gpu


def _instances():
    sweep = synth.cfg2_argon_sweep()
    mix = synth.configs.mixture_ar_co2()
    cfgs = [sweep[0], sweep[12], sweep[31],
            synth.SwarmConfig(mix, synth.td_to_field(50.0), B_T=1.0, B_angle_rad=0.7),
            synth.SwarmConfig(synth.cfg4_mixtures()[3], synth.td_to_field(300.0)),
            synth.cfg1_maxwell()]
    jobs = [(1500, 300, 0), (700, 900, 1), (2100, 150, 2), (999, 400, 3), (64, 2000, 4), (3000, 100, 5)]
    return cfgs, jobs


def _same(a, b):
    assert len(a) == len(b)
    for f in a.dtype.names:
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_batch_equals_single_runs(gpu, precision):
    sw = gpu
    cfgs, jobs = _instances()
    singles = []
    for cfg, (ne, nc, seed) in zip(cfgs, jobs):
        s = sw.Swarm.from_config(cfg, precision)
        s.run(ne, nc, seed)
        singles.append((s.records(), s.tallies()))
    hs = [sw.Swarm.from_config(c, precision) for c in cfgs]
    # the default shape, one electron per lane and item, large items, and items of 8 per lane
    # whose last share is cut into items of 2 per lane
    variants = [dict(), dict(block_size=128, chunk=128, pending_trigger=1),
                dict(block_size=512, chunk=512 * 16, pending_trigger=64, use_graph=1),
                dict(block_size=256, chunk=256 * 8, pending_trigger=40)]
    for opts in variants:
        sw.swarm_batch_run([h.h for h in hs], jobs, opts)
        for h, (rec, tal) in zip(hs, singles):
            _same(h.records(), rec)
            assert h.tallies() == tal


def test_graph_replays_are_identical(gpu):
    sw = gpu
    cfgs, jobs = _instances()
    hs = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in cfgs]
    b = sw.swarm_batch_create([h.h for h in hs], jobs, dict(use_graph=1))
    try:
        outs = []
        for _ in range(3):
            sw.swarm_batch_launch(b)
            sw.swarm_batch_wait(b)
            outs.append([sw.swarm_batch_tallies(b, i) for i in range(len(hs))])
            outs[-1].append(hs[2].records().copy())
        for o in outs[1:]:
            for i in range(len(hs)):
                assert o[i] == outs[0][i]
            _same(o[-1], outs[0][-1])
    finally:
        sw.swarm_batch_destroy(b)


def test_batch_fp64_matches_oracle(gpu):
    sw = gpu
    cfgs, jobs = _instances()
    hs = [sw.Swarm.from_config(c, sw.SWARM_FP64) for c in cfgs]
    sw.swarm_batch_run([h.h for h in hs], jobs, dict(use_graph=1))
    for h, cfg, (ne, nc, seed) in zip(hs, cfgs, jobs):
        r = oracle.OracleModel.from_config(cfg).run(ne, nc, seed)
        compare_records(h.records(), r.records)


def test_autotune_returns_valid_options(gpu):
    sw = gpu
    cfgs, jobs = _instances()
    hs = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in cfgs]
    best = sw.swarm_autotune([h.h for h in hs], jobs, 100)
    assert best["block_size"] in (128, 256, 512)
    assert 1 <= best["pending_trigger"] <= 64
    assert best["chunk"] % best["block_size"] == 0


def test_batch_rejects_real_mode_and_mixed_precision(gpu):
    sw = gpu
    a = sw.Swarm.from_config(synth.cfg1_maxwell(), sw.SWARM_FP64)
    b = sw.Swarm.from_config(synth.cfg1_maxwell(), sw.SWARM_FP32_MIXED)
    with pytest.raises(sw.SwarmError):
        sw.swarm_batch_run([a.h, b.h], [(10, 10, 0), (10, 10, 1)])
    c = sw.Swarm.from_config(synth.cfg3_mixture_real(), sw.SWARM_FP64)
    with pytest.raises(sw.SwarmError):
        sw.swarm_batch_run([c.h], [(10, 10, 0)])


def test_reordered_launches_give_the_same_bits(gpu):
    """After its first launch a batch orders its items by each instance's measured work per
    electron; the launches after it, in that order, give the bits of the first (instances
    listed fast ones first, so the order does change)."""
    sw = gpu
    cfgs = list(reversed(synth.cfg2_argon_sweep()))[::4]
    jobs = [(20000, 500, 3 + i) for i in range(len(cfgs))]
    hs = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in cfgs]
    b = sw.swarm_batch_create([h.h for h in hs], jobs, {"use_graph": 1})
    try:
        sw.swarm_batch_launch(b)
        sw.swarm_batch_wait(b)
        first = [h.records().tobytes() for h in hs]
        for _ in range(2):
            sw.swarm_batch_launch(b)
            sw.swarm_batch_wait(b)
            assert [h.records().tobytes() for h in hs] == first
    finally:
        sw.swarm_batch_destroy(b)
