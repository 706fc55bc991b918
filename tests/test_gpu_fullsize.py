"""Parity at the workloads' full sizes, in the launch configuration the benchmark uses,
on outputs the oracle can compute one by one (sampled electrons and whole lineages), and
through size-independent properties (FP32 against FP64 tallies, counts)."""
import math

import numpy as np
import pytest

import oracle
import synth
from swarm_testutil import compare_records, sort_by_id, tally_agreement

pytestmark = pytest.mark.gpu

QE, ME = 1.602176634e-19, 9.1093837015e-31


def _oracle_one(cfg, eid, n_c, seed):
    """The oracle's record of one primary (and its lineage) computed on its own."""
    return oracle.OracleModel.from_config(cfg).run(1, n_c, seed, n_threads=1, first_id=eid).records


def test_argon_sweep_full_size_fp64_samples_and_fp32_agreement(gpu):
    """The benchmark workload (32 x 1e5 electrons x 2e4 collisions): FP64 batched records of
    sampled electrons equal the oracle's, and every FP32 tally agrees with FP64."""
    sw = gpu
    cfgs = synth.cfg2_argon_sweep()
    jobs = [(c.n_electrons, c.n_collisions, c.seed) for c in cfgs]
    h64 = [sw.Swarm.from_config(c, sw.SWARM_FP64) for c in cfgs]
    sw.swarm_batch_run([h.h for h in h64], jobs, {"use_graph": 1})
    rng = np.random.default_rng(0)
    for i in (0, 9, 20, 31):
        rec = sort_by_id(h64[i].records())
        assert len(rec) == 100_000 and np.all(rec["flags"] == 1)
        for eid in rng.choice(100_000, 3, replace=False):
            ref = _oracle_one(cfgs[i], int(eid), 20_000, 0)
            compare_records(rec[int(eid):int(eid) + 1], ref)
    t64 = [h.tallies() for h in h64]
    h32 = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in cfgs]
    sw.swarm_batch_run([h.h for h in h32], jobs, {"use_graph": 1})
    t32 = [h.tallies() for h in h32]
    for a, b in zip(t32, t64):
        assert a["n_real"] == b["n_real"] == 100_000 * 20_000
        bad = tally_agreement(a, b, keys=["W", "mean_energy", "mean_energy_after", "D", "DL", "DT", "sigma",
                                          "alpha"])
        assert not bad, bad


def test_mixture_real_secondaries_full_electron_count(gpu):
    """1e6 primaries of the 90:10 mixture at 100 Td, 1 T at 45 degrees, real secondaries,
    with the largest collision budget whose lineage growth fits the default capacity:
    whole lineages of sampled primaries equal the oracle's."""
    sw = gpu
    cfg = synth.cfg3_mixture_real(n_collisions=2000)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.run(cfg.n_electrons, cfg.n_collisions, 0)
    T = s.tallies()
    assert T["n_dropped"] == 0
    assert T["n_created"] > 5 * cfg.n_electrons
    rec = sort_by_id(s.records())
    assert len(rec) == T["n_electrons"]
    for eid in (0, 1, 777, 123456, 999_999):
        ref = _oracle_one(cfg, eid, cfg.n_collisions, 0)
        idx = np.searchsorted(rec["id"], ref["id"])
        assert np.array_equal(rec["id"][idx], ref["id"])
        compare_records(rec[idx], ref)
    s32 = sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED)
    s32.run(cfg.n_electrons, cfg.n_collisions, 0)
    T32 = s32.tallies()
    bad = tally_agreement(T32, T, keys=["W", "Wx", "Wy", "mean_energy", "D_vec", "alpha"])
    assert not bad, bad
    assert abs(T32["n_electrons"] / T["n_electrons"] - 1) < 0.02


def test_mixture_real_secondaries_stated_budget_reports_capacity(gpu):
    """At the stated 5e4 collisions the lineages would grow as exp(85): the run stops early
    with SWARM_ERR_CAPACITY instead of dropping electrons silently."""
    sw = gpu
    cfg = synth.cfg3_mixture_real()
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED)
    with pytest.raises(sw.SwarmError) as ei:
        s.run(cfg.n_electrons, cfg.n_collisions, 0)
    assert ei.value.status == sw.SWARM_ERR_CAPACITY
    T = s.tallies()
    assert T["n_dropped"] > 0


def test_batch_256_instances_full_size(gpu):
    """The 256-instance sweep (4 mixtures x 64 E/N, B = 0 or 1 T, uneven sizes) in one
    persistent FP32 launch; sampled instances against FP64 single runs and the oracle."""
    sw = gpu
    cfgs = synth.cfg4_batch()
    jobs = [(c.n_electrons, c.n_collisions, c.seed) for c in cfgs]
    h32 = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in cfgs]
    sw.swarm_batch_run([h.h for h in h32], jobs, {"use_graph": 1})
    t32 = [h.tallies() for h in h32]
    for c, t in zip(cfgs, t32):
        assert t["n_real"] == c.n_electrons * c.n_collisions
        assert t["n_finished"] == c.n_electrons
    work = np.array([ne * nc for ne, nc, _ in jobs], dtype=float)
    cheap = [i for i in np.argsort(work) if work[i] < 2e9]
    sample = cheap[::max(1, len(cheap) // 10)][:10]
    for i in sample:
        c = cfgs[i]
        s = sw.Swarm.from_config(c, sw.SWARM_FP64)
        s.run(*jobs[i])
        t64 = s.tallies()
        bad = tally_agreement(t32[i], t64, keys=["W", "Wx", "Wy", "mean_energy", "D_vec", "alpha"])
        assert not bad, (i, c.label, bad)
        rec = sort_by_id(s.records())
        eid = int(c.n_electrons // 2)
        compare_records(rec[eid:eid + 1], _oracle_one(c, eid, c.n_collisions, c.seed))
