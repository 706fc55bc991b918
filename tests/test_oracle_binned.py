"""Pins of the oracle's binned trial frequency (section "Trial frequency strategies": the
BinnedTrialFrequency, b bins per decade of energy, each with the largest collision
frequency in it; after a fail a retry with the largest frequency of the bins between, and a
second fail where the paper throws).

  * the bin of every grid node, against exact integer arithmetic (node^b against 10^k);
  * every bin's nu' bounds the interpolated rate on dense samples of its cells and equals
    the largest end-node rate of those cells, raised by 2^-20;
  * closed forms: a constant-rate gas runs with nu' = nu (1 + 2^-20), never fails, and keeps
    the drift velocity eE/(m nu); without a field and with infinitely heavy targets no
    electron changes its bin, so nothing fails;
  * brute force: a plain-Python run of the strategy's steps for a few electrons, built on
    the oracle's primitives (streams, motion, rate lookup, channel choice, energy transfer)
    but not on its loop, gives the same records.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies

QE, ME, AMU = oracle.constants()


def exact_bin(eps, b):
    """floor(b log10 eps) for an exactly representable eps, by comparing eps^b with 10^k."""
    q = Fraction(eps) ** b
    k = math.floor(b * math.log10(eps))
    while Fraction(10) ** (k + 1) <= q:
        k += 1
    while Fraction(10) ** k > q:
        k -= 1
    return k


def _model(cfg, bins=10, grace=5000, **kw):
    return oracle.OracleModel.from_config(cfg.scaled(trial_strategy=2, trial_bins=bins, trial_grace=grace), **kw)


@pytest.mark.parametrize("b", [1, 3, 10, 64, 100])
def test_node_bins_exact(b):
    m = _model(synth.cfg2_argon_sweep()[12], bins=b)
    nodes, _ = m.tables()
    node_bin, nup = m.bins()
    ks = np.array([exact_bin(float(e), b) for e in nodes])
    np.testing.assert_array_equal(node_bin, ks - ks[0])
    assert len(nup) == ks[-1] - ks[0] + 1
    # 1, 10, 100 and 1000 eV are grid nodes and open their bins
    for d in range(4):
        g = int(np.flatnonzero(nodes == 10.0 ** d)[0])
        assert node_bin[g] == node_bin[g - 1] + 1


@pytest.mark.parametrize("b,i", [(10, 3), (10, 31), (4, 18), (37, 25)])
def test_bin_nup_is_the_bin_maximum(b, i):
    cfg = synth.cfg2_argon_sweep()[i]
    m = _model(cfg, bins=b)
    nodes, _ = m.tables()
    node_bin, nup = m.bins()
    G = len(nodes)
    top = np.zeros(len(nup))
    ws = np.linspace(0.0, 1.0, 9, endpoint=False)
    for g in range(G):
        k = node_bin[g]
        if g + 1 < G:
            # samples inside the cell [node g, node g+1)
            for w in ws:
                eps = nodes[g] + w * (nodes[g + 1] - nodes[g])
                nu, _ = m.nu_grid(eps)
                assert nu <= nup[k], (g, w, nu, nup[k])
            ends = (m.nu_grid(nodes[g])[0], m.nu_grid(nodes[g + 1])[0])
        else:
            ends = (m.nu_grid(nodes[g])[0], m.nu_grid(2.0 * nodes[g])[0])
        top[k] = max(top[k], *ends)
    # below the grid and above its top: the end bins
    assert m.nu_grid(0.5 * nodes[0])[0] <= nup[0]
    assert m.nu_grid(10 * nodes[-1])[0] <= nup[-1]
    np.testing.assert_array_equal(nup, np.minimum((1.0 + 2.0 ** -20) * top, m.majorant))
    assert nup.max() == m.majorant     # the bin of the table maximum holds the constant nu'


def test_constant_rate_gas_never_fails():
    # nu = 1e12 at every energy: every bin's nu' is nu (1 + 2^-20), far below the fixed
    # constant value 4e12, so almost every trial is real and nothing fails.
    cfg = synth.cfg1_maxwell(n_electrons=3000, n_collisions=2000).scaled(
        user_majorant=4e12, trial_strategy=2, trial_bins=10, trial_grace=50)
    T = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 1).records)
    assert T["n_fail"] == 0
    assert T["efficiency"] > 1 - 1e-4
    W = QE * synth.td_to_field(10.0) / (ME * 1e12)
    assert abs(T["W"][0] - W) < 3.5 * T["W"][1]


def test_no_field_heavy_targets_never_fail():
    comp = synth.random_component(np.random.default_rng(9), fraction=1.0, max_inelastic=0)
    comp = synth.Component(1e12, 1.0, [ch for ch in comp.channels if ch.kind == synth.ELASTIC])
    cfg = synth.SwarmConfig([comp], 0.0, init_energy_eV=3.0, n_electrons=400, n_collisions=500,
                            trial_strategy=2, trial_bins=50, trial_grace=1)
    T = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 2).records)
    assert T["n_fail"] == 0


def test_binned_fails_and_is_more_efficient():
    cfg = synth.cfg2_argon_sweep(n_electrons=1500, n_collisions=1500)[10]
    a = tallies(oracle.OracleModel.from_config(cfg).run(cfg.n_electrons, cfg.n_collisions, 0).records)
    r = _model(cfg, bins=10, grace=5000).run(cfg.n_electrons, cfg.n_collisions, 0).records
    b = tallies(r)
    assert b["n_real"] == a["n_real"]
    assert b["efficiency"] > 1.5 * a["efficiency"]
    assert b["n_fail"] > 0
    trials = b["n_real"] + b["n_null"] + b["n_forbidden"] + b["n_fail"]
    assert abs(b["efficiency"] - b["n_real"] / trials) < 1e-15
    # some retries fail again (flag 16); those electrons still finish
    flagged = (r["flags"] & oracle.FLAG_RETRY_FAILED) != 0
    assert flagged.any()
    assert np.all(r["flags"][flagged] & oracle.FLAG_FINISHED)


def test_invalid_binned_refused():
    cfg = synth.cfg2_argon_sweep()[3]
    for bins, grace in ((0, 10), (101, 10), (10, 0)):
        with pytest.raises(ValueError):
            _model(cfg, bins=bins, grace=grace)


# ---- brute force ------------------------------------------------------------------------

def _iso(u_cos, u_phi):
    ct = 1.0 - 2.0 * u_cos
    st = math.sqrt(max(0.0, (1.0 - ct) * (1.0 + ct)))
    ph = 2.0 * math.pi * u_phi
    return np.array([st * math.cos(ph), st * math.sin(ph), ct])


def _energy(v):
    return 0.5 * ME * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / QE


def _speed(eps):
    return math.sqrt(2.0 * eps * QE / ME)


def brute_force(m, cfg, b, grace0, eid, n_coll, seed):
    """One electron (B = 0, dummy secondaries, isotropic scattering) with the binned trial
    frequency, step by step: renewal after `grace0` trials from the current energy's bin,
    a fail (nu > nu') back to the last real collision with the largest nu' of the bins from
    the anchor's to the failing energy's, a second fail before the next real collision or
    renewal (flag 16) with the constant nu'."""
    nodes, C = m.tables()
    F = C[-1]
    G = len(nodes)
    ks = [exact_bin(float(e), b) for e in nodes]
    kb = [k - ks[0] for k in ks]
    top = [0.0] * (kb[-1] + 1)
    for g in range(G):
        cell = max(F[g], F[g + 1]) if g + 1 < G else F[g]
        top[kb[g]] = max(top[kb[g]], cell)
    cap = m.majorant
    bin_nup = [min((1.0 + 2.0 ** -20) * t, cap) for t in top]

    def bin_of(eps):
        if eps < nodes[0]:
            return kb[0]
        if eps >= nodes[-1]:
            return kb[-1]
        g = int(np.searchsorted(nodes, eps, side="right")) - 1
        return kb[g]

    h = oracle.stream_block(seed, eid, oracle.INIT_HI, 0)
    l = oracle.stream_block(seed, eid, oracle.INIT_LO, 0)
    v = _iso(oracle.uniform53(h[0], l[0]), oracle.uniform53(h[1], l[1])) * _speed(cfg.init_energy_eV)
    r = np.zeros(3)
    t = 0.0
    T = 0.0
    k = 0
    nup = bin_nup[bin_of(cfg.init_energy_eV)]
    grace = grace0
    retry = False
    rec = dict(flags=0, n_null=0, n_fail=0, n_forbidden=0, n_over=0, G=0, D=0, blocks=0,
               sum_eps=0.0, sum_epsp=0.0)
    block = 0
    while k < n_coll:
        hi = oracle.stream_block(seed, eid, oracle.TRIAL_HI, block)
        lo = oracle.stream_block(seed, eid, oracle.TRIAL_LO, block)
        block += 1
        for sub in (0, 1):
            u_f = oracle.uniform53(hi[2 * sub], lo[2 * sub])
            u_r = oracle.uniform53(hi[2 * sub + 1], lo[2 * sub + 1])
            T += -math.log(1.0 - u_f) / nup
            _, vT = m.move(r, v, T)
            eps = _energy(vT)
            nu, over = m.nu_grid(eps)
            if nu > nup:                                   # fail
                rec["n_fail"] += 1
                T = 0.0
                if retry:
                    rec["flags"] |= oracle.FLAG_RETRY_FAILED
                    nup = cap
                else:
                    a, f = bin_of(_energy(v)), bin_of(eps)
                    nup = max(bin_nup[min(a, f):max(a, f) + 1])
                retry = True
                grace = grace0
                break
            x = u_r * nup
            c = m.select(eps, x)
            if c < 0:                                      # null
                rec["n_null"] += 1
                grace -= 1
                if grace == 0:
                    nup, grace, retry = bin_nup[bin_of(eps)], grace0, False
                continue
            _, kind, thr, mass = m.channel_info[c]
            M = mass * AMU
            if kind in (synth.EXCITATION, synth.IONIZATION) and eps < thr * ((ME + M) / M):
                rec["n_forbidden"] += 1                    # treated as null
                grace -= 1
                if grace == 0:
                    nup, grace, retry = bin_nup[bin_of(eps)], grace0, False
                break
            if over:
                rec["n_over"] += 1
            rT, _ = m.move(r, v, T)
            sh = oracle.stream_block(seed, eid, oracle.SCAT_HI, k)
            sl = oracle.stream_block(seed, eid, oracle.SCAT_LO, k)
            n = _iso(oracle.uniform53(sh[0], sl[0]), oracle.uniform53(sh[1], sl[1]))
            v2 = vT[0] * vT[0] + vT[1] * vT[1] + vT[2] * vT[2]
            cos_t = (n[0] * vT[0] + n[1] * vT[1] + n[2] * vT[2]) / math.sqrt(v2)
            epsp = max(oracle.energy_after(kind, eps, thr, cos_t, mass), 0.0)
            rec["sum_eps"] += eps
            if kind == synth.IONIZATION:
                epsp *= 0.5
                rec["G"] += 1
            elif kind == synth.ATTACHMENT:
                rec["D"] += 1
            rec["sum_epsp"] += epsp
            k += 1
            r = rT
            t += T
            T = 0.0
            v = n * _speed(epsp)
            retry = False
            grace -= 1
            if grace == 0:
                nup, grace, retry = bin_nup[bin_of(epsp)], grace0, False
            break
    rec.update(flags=rec["flags"] | oracle.FLAG_FINISHED, k_end=k, blocks=block, r=r, t=t)
    return rec


@pytest.mark.parametrize("i,b,grace", [(0, 30, 50), (21, 10, 7), (31, 4, 300), (31, 20, 1)])
def test_brute_force_records(i, b, grace):
    cfg = synth.cfg2_argon_sweep()[i]
    m = _model(cfg, bins=b, grace=grace)
    n_e, n_c, seed = 4, 250, 13
    got = m.run(n_e, n_c, seed).records
    total_fail = 0
    for e in range(n_e):
        want = brute_force(m, cfg, b, grace, e, n_c, seed)
        g = got[got["id"] == e][0]
        for key in ("flags", "n_null", "n_fail", "n_forbidden", "n_over", "G", "D", "blocks", "k_end"):
            assert int(g[key]) == int(want[key]), (e, key, int(g[key]), want[key])
        np.testing.assert_allclose(g["r"], want["r"], rtol=1e-12, atol=1e-18)
        for key in ("t", "sum_eps", "sum_epsp"):
            assert g[key] == pytest.approx(want[key], rel=1e-12), key
        total_fail += want["n_fail"]
    assert total_fail > 0
