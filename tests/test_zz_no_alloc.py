"""swarm_run_noalloc, the entry point for callers that cannot allocate device memory: through
the C ABI, records written to a caller buffer and tallies equal those of swarm_run on the same
inputs, bit for bit, on two calls in a row (the second smaller, so that the shared scratch
array holds the first call's contents), and the FP64 records equal the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from swarm_testutil import compare_records

pytestmark = pytest.mark.gpu


def _noalloc(sw, s, n_e, n_c, seed):
    import torch
    buf = torch.empty(n_e * sw.RECORD_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    sw.swarm_run_noalloc(s.h, n_e, n_c, seed, buf.data_ptr())
    rec = buf.cpu().numpy().view(sw.RECORD_DTYPE)
    return rec, s.tallies()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_noalloc_equals_swarm_run(gpu, precision):
    sw = gpu
    cfg = synth.cfg3_mixture_real().scaled(secondaries=0)     # argon:CO2, 1 T at 45 deg, 28 channels
    s = sw.Swarm.from_config(cfg, precision)
    ref = sw.Swarm.from_config(cfg, precision)
    for n_e, n_c, seed in ((20011, 300, 4), (777, 200, 9)):   # ragged sizes, the second smaller
        rec, T = _noalloc(sw, s, n_e, n_c, seed)
        ref.run(n_e, n_c, seed)
        want = ref.records()
        assert rec.tobytes() == want.tobytes()
        assert T == ref.tallies()
        if precision == sw.SWARM_FP64 and n_e < 1000:
            compare_records(rec, oracle.OracleModel.from_config(cfg).run(n_e, n_c, seed).records)
    with pytest.raises(sw.SwarmError) as ei:
        s.records()                # the records are in the caller's buffer
    assert ei.value.status == sw.SWARM_ERR_STATE


def test_noalloc_refuses_what_it_cannot_hold(gpu):
    sw = gpu
    cfg = synth.cfg2_argon_sweep()[5]
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP32_MIXED)
    with pytest.raises(sw.SwarmError) as ei:
        sw.swarm_run_noalloc(s.h, (1 << 22) + 1, 10, 0, 1 << 40)    # refused before any device work
    assert ei.value.status == sw.SWARM_ERR_INVALID_ARG
    real = sw.Swarm.from_config(synth.cfg3_mixture_real(n_electrons=10, n_collisions=10), sw.SWARM_FP32_MIXED)
    with pytest.raises(sw.SwarmError) as ei:
        sw.swarm_run_noalloc(real.h, 10, 10, 0, 1 << 40)
    assert ei.value.status == sw.SWARM_ERR_INVALID_ARG
