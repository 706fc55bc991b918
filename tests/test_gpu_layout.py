"""LDS table layouts and launch options change the schedule only: the running sums staged in
LDS (table layout 1) give the same bits as reading them through L2, for batches, single
runs and real secondaries; the autotuner returns options that run."""
import numpy as np
import pytest

import oracle
import synth
from swarm_testutil import compare_records

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_table_layout_1_equals_layout_0(gpu, precision):
    sw = gpu
    base = synth.cfg2_argon_sweep()
    cfgs = [base[3], base[16], base[29], base[16].scaled(trial_strategy=1),
            base[22].scaled(components=[c.with_scattering(1) for c in base[22].components])]
    jobs = [(2000 + 100 * i, 400, 7 + i) for i in range(len(cfgs))]
    ref = [sw.Swarm.from_config(c, precision) for c in cfgs]
    sw.swarm_batch_run([h.h for h in ref], jobs, {})
    for shape in ({"table_layout": 1}, {"table_layout": 1, "block_size": 256, "service_waves": 1}):
        hs = [sw.Swarm.from_config(c, precision) for c in cfgs]
        sw.swarm_batch_run([h.h for h in hs], jobs, shape)
        for a, b in zip(ref, hs):
            assert a.records().tobytes() == b.records().tobytes(), shape


def test_table_layout_1_single_and_real_runs(gpu):
    sw = gpu
    # argon-like (5 channels) fits in LDS; real secondaries with an argon-like gas
    cfg = synth.cfg2_argon_sweep()[28]
    a = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    a.run(3000, 300, 4)
    b = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    b.set_launch_opts({"table_layout": 1})
    b.run(3000, 300, 4)
    assert a.records().tobytes() == b.records().tobytes()
    real = synth.cfg3_mixture_real(n_electrons=64, n_collisions=900).scaled(components=[synth.argon_like()])
    r = sw.Swarm.from_config(real, sw.SWARM_FP64)
    r.set_launch_opts({"table_layout": 1, "block_size": 64})
    r.run(64, 900, 2)
    compare_records(r.records(), oracle.OracleModel.from_config(real).run(64, 900, 2).records)


def test_table_layout_1_falls_back_when_tables_do_not_fit(gpu):
    # the Ar/CO2 mixture's running sums (28 channels) exceed a work-group's LDS
    sw = gpu
    cfg = synth.cfg3_mixture_real().scaled(secondaries=0)
    a = sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED)
    sw.swarm_batch_run([a.h], [(1500, 300, 1)], {"table_layout": 1})
    b = sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED)
    sw.swarm_batch_run([b.h], [(1500, 300, 1)], {})
    assert a.records().tobytes() == b.records().tobytes()


def test_autotune_returns_runnable_options(gpu):
    sw = gpu
    cfgs = synth.cfg2_argon_sweep(n_electrons=20000, n_collisions=500)[::8]
    hs = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in cfgs]
    jobs = [(c.n_electrons, c.n_collisions, c.seed) for c in cfgs]
    best = sw.swarm_autotune([h.h for h in hs], jobs, 100)
    assert best["block_size"] in (128, 256, 512) and best["table_layout"] in (0, 1)
    sw.swarm_batch_run([h.h for h in hs], jobs, best)
    ref = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in cfgs]
    sw.swarm_batch_run([h.h for h in ref], jobs, {})
    for a, b in zip(hs, ref):
        assert a.records().tobytes() == b.records().tobytes()
