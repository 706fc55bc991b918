"""Real secondaries: a launch parks its last few running electrons (each at its next real
collision) for the next launch once it has created enough secondaries.  That changes the
schedule only: runs that park eagerly, by default or never give the same records, and parked
lineages equal the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from swarm_testutil import compare_records, sort_by_id

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_parking_changes_no_record(gpu, precision):
    sw = gpu
    cfg = synth.cfg3_mixture_real(n_electrons=200_000, n_collisions=1000)
    out = {}
    for park in (-1, 0, 64):     # never, the default (32 lanes), any wave with a running lane
        s = sw.Swarm.from_config(cfg, precision)
        s.set_launch_opts({"park_lanes": park})
        s.run(cfg.n_electrons, cfg.n_collisions, 3)
        T = s.tallies()
        assert T["n_dropped"] == 0
        out[park] = (sort_by_id(s.records()), T["n_real"], s.launches())
    parked_never = out[-1][2][1]
    assert parked_never == 0
    assert out[64][2][1] > 0, "the eager setting parked nothing"
    for park in (0, 64):
        assert out[park][1] == out[-1][1]
        assert out[park][0].tobytes() == out[-1][0].tobytes(), park


def test_parking_changes_no_traced_event(gpu):
    """The traced kernel parks too: the event sequences of primaries claimed first and last
    (the last ones run in the waves that park) are the same with eager parking as without."""
    sw = gpu
    cfg = synth.cfg3_mixture_real(n_electrons=200_000, n_collisions=1000)
    ids = [0, 1, 100_000] + list(range(199_990, 200_000))
    out = {}
    for park in (-1, 64):
        s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
        s.set_launch_opts({"park_lanes": park})
        s.set_trace(ids, 2048)
        s.run(cfg.n_electrons, cfg.n_collisions, 3)
        ev, counts = s.trace_events()
        out[park] = (ev.tobytes(), counts.tolist(), s.launches()[1])
    assert out[64][2] > 0
    assert out[64][1] == out[-1][1]
    assert out[64][0] == out[-1][0]


def test_parked_lineages_equal_the_oracle(gpu):
    """Eager parking on a run of 50,000 primaries: the whole lineages of sampled primaries
    equal the oracle's records, each lineage computed on its own."""
    sw = gpu
    cfg = synth.cfg3_mixture_real(n_electrons=50_000, n_collisions=800)
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64)
    s.set_launch_opts({"park_lanes": 64})
    s.run(cfg.n_electrons, cfg.n_collisions, 5)
    launches, parked = s.launches()
    assert parked > 0
    rec = sort_by_id(s.records())
    for pid in (0, 4321, 49_999):
        ref = sort_by_id(oracle.OracleModel.from_config(cfg).run(1, cfg.n_collisions, 5, n_threads=1,
                                                                 first_id=pid).records)
        idx = np.searchsorted(rec["id"], ref["id"])
        assert np.array_equal(rec["id"][idx], ref["id"])
        compare_records(rec[idx], ref)
