"""Random combinations of every option on random gases (the request generator's mixtures):
trial strategy (constant, variable, binned with random grace, zeta and bins), scattering model
per component (isotropic, screened Coulomb, constant xi), moving targets at a random
temperature, the relativistic mover, B on or off, dummy or real secondaries.  For each, the
FP64 records of the GPU equal the oracle's element by element (R22), so interactions between
the options are covered beyond the tests of each option alone."""
import numpy as np
import pytest

import oracle
import synth
from swarm_testutil import compare_records

pytestmark = pytest.mark.gpu


def random_case(i):
    rng = np.random.default_rng([77, i])
    base = synth.cfg5_request(100 + i, max_components=3)
    comps = []
    for c in base.components:
        model = int(rng.integers(0, 3))
        if model == 1:
            comps.append(c.with_scattering(1))
        elif model == 2:
            comps.append(c.with_scattering(2, float(rng.uniform(0.2, 1.0))))
        else:
            comps.append(c)
    # every fourth case takes the relativistic mover with B (its most involved path)
    thermal = int(i % 4 != 3 and rng.random() < 0.4)
    relativistic = int(i % 4 == 3 or (not thermal and rng.random() < 0.35))
    keep_b = i % 4 == 3 or rng.random() < 0.6
    return base.scaled(components=comps, B_T=base.B_T if keep_b else 0.0,
                       trial_strategy=int(rng.integers(0, 3)), trial_grace=int(rng.choice([1, 37, 500])),
                       trial_bins=int(rng.choice([3, 10, 40])), trial_zeta=float(rng.uniform(0.1, 1.0)),
                       thermal_targets=thermal, T_K=float(rng.uniform(50.0, 3000.0)),
                       relativistic=relativistic, secondaries=int(rng.random() < 0.3),
                       label=f"random-{i}")


def _describe(cfg):
    return (f"{cfg.label}: strategy {cfg.trial_strategy}, scattering {[c.scattering for c in cfg.components]}, "
            f"thermal {cfg.thermal_targets}, relativistic {cfg.relativistic}, B {cfg.B_T:.2f}, "
            f"secondaries {cfg.secondaries}")


@pytest.mark.parametrize("i", range(16))
def test_fp64_records_random_options(gpu, i):
    sw = gpu
    cfg = random_case(i)
    n_e, n_c, seed = 200, 150, 3 + i
    print(_describe(cfg), flush=True)
    cap = 200_000            # real secondaries can avalanche on these gases
    s = sw.Swarm.from_config(cfg, sw.SWARM_FP64, capacity=cap)
    s.run(n_e, n_c, seed)
    r = oracle.OracleModel.from_config(cfg).run(n_e, n_c, seed, capacity=cap)
    assert r.status == 0
    compare_records(s.records(), r.records)


def test_random_options_cover_every_option():
    """The cases above draw every option at least once."""
    cases = [random_case(i) for i in range(16)]
    assert {c.trial_strategy for c in cases} == {0, 1, 2}
    assert {m for c in cases for m in (k.scattering for k in c.components)} == {0, 1, 2}
    assert any(c.thermal_targets for c in cases) and any(c.relativistic for c in cases)
    assert any(c.relativistic and c.B_T > 0 for c in cases)
    assert any(c.secondaries for c in cases) and any(c.B_T == 0 for c in cases)
