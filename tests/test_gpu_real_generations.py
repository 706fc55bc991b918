"""Real-secondaries mode runs in generations: one launch for the primaries, then one for the
secondaries each generation created.  The per-electron results do not depend on the launch
shape.  After an overflow of the secondary queue every electron that was created has a
record: those that finished before it equal the oracle's (whose run has no capacity limit),
those stopped by it are a prefix of the oracle's history (flag 8), and those never started
carry flag 8 with no collision made."""
import numpy as np
import pytest

import oracle
import synth
from swarm_testutil import compare_records, sort_by_id

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_real_records_independent_of_launch_shape(gpu, precision):
    sw = gpu
    prec = sw.SWARM_FP64 if precision == "fp64" else sw.SWARM_FP32_MIXED
    n_e, n_c, seed = 3000, 1500, 6
    cfg = synth.cfg3_mixture_real(n_electrons=n_e, n_collisions=n_c)
    ref = None
    for opts in ({}, {"block_size": 64, "pending_trigger": 1}, {"block_size": 512, "pending_trigger": 64},
                 {"block_size": 256, "table_layout": 1}):
        s = sw.Swarm.from_config(cfg, prec)
        if opts:
            s.set_launch_opts(opts)
        s.run(n_e, n_c, seed)
        rec = sort_by_id(s.records())
        if ref is None:
            ref = rec
            assert len(rec) > 2 * n_e          # secondaries of several generations
        else:
            assert rec.tobytes() == ref.tobytes(), opts


def test_overflow_records_every_created_electron(gpu):
    sw = gpu
    n_e, n_c, seed, cap = 400, 3000, 9, 4400
    cfg = synth.cfg3_mixture_real(n_electrons=n_e, n_collisions=n_c)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64, capacity=cap)
    with pytest.raises(sw.SwarmError) as ei:
        s.run(n_e, n_c, seed)
    assert ei.value.status == sw.SWARM_ERR_CAPACITY
    T = s.tallies()
    rec = sort_by_id(s.records())
    assert len(rec) == cap and T["n_electrons"] == cap and T["n_dropped"] > 0
    assert len(np.unique(rec["id"])) == cap
    assert np.array_equal(rec["id"][:n_e], np.arange(n_e, dtype=np.uint64))   # every primary

    full = sort_by_id(oracle.OracleModel.from_config(cfg).run(n_e, n_c, seed).records)
    idx = np.searchsorted(full["id"], rec["id"])
    assert np.all(idx < len(full)) and np.array_equal(full["id"][np.minimum(idx, len(full) - 1)], rec["id"])
    ref = full[idx]
    stopped = (rec["flags"] & 8) != 0
    # finished or attached before the overflow: the oracle's records, element by element
    compare_records(rec[~stopped], ref[~stopped])
    assert np.count_nonzero(~stopped & (rec["id"] >= np.uint64(1 << 63))) > 0   # secondaries among them
    # stopped by the overflow: a prefix of the same history
    assert np.all(rec["k_start"][stopped] == ref["k_start"][stopped])
    assert np.all(rec["k_end"][stopped] <= ref["k_end"][stopped])
    # never started: recorded as created
    unstarted = stopped & (rec["blocks"] == 0)
    assert unstarted.any()
    assert np.all(rec["k_end"][unstarted] == rec["k_start"][unstarted])
    assert np.all(rec["n_null"][unstarted] == 0)
