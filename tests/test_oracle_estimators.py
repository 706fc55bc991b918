"""Pins of the swarm-tally estimators of section 'Determination of swarm attributes' that the
closed-form runs of test_oracle_swarm.py leave open: the per-electron (paper-form) Townsend
coefficients <alpha> = (1/N) sum G_n/z_n and <eta> = (1/N) sum D_n/z_n, and the vector form of
the displacement family (d_n = x_n - t_n W_vec; D, D_L, D_T, sigma of it).

Each test checks oracle/tallies.py against something other than its own formulas: a process
whose answer is known (constant rates, a random walk written independently in numpy), or an
exact property of the estimators (a uniform drift added to every electron)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle.tallies import tallies

QE, ME, AMU = oracle.constants()
K = synth.tables.MAXWELL_K
NU = 1e12          # the constant-rate components' total rate at N = 2.5e25 (their k sums to K)


def _within(val, want, sig, k=4.0):
    assert abs(val - want) <= k * sig, (val, want, sig, (val - want) / sig)


# ---- Townsend coefficients, paper form ------------------------------------------------

@pytest.fixture(scope="module")
def light_target_run():
    # Constant rates nu_el : nu_i : nu_a = 0.80 : 0.15 : 0.05 of NU, dummy ionisation and
    # attachment, on a light target (0.01 u).  The light target loses about a tenth of the
    # energy per collision, so the swarm stays cold and every electron's drift length z_n
    # after n = 4000 collisions lies within about 5% of its mean: the mean of the ratios
    # G_n/z_n is then close to the ratio of the means.
    comp = synth.constant_rate_component(0.01, 1.0, 0.80 * K, 0.15 * K, 0.05 * K)
    E = synth.td_to_field(30.0)
    rec = oracle.OracleModel([comp], E).run(4000, 4000, 11).records
    return rec, tallies(rec)


def _ratio_mean_bias(z):
    # E[c/z] = (c/E[z]) (1 + Var(z)/E[z]^2 + O(n^-2)) for a drift length z_n that is the sum
    # of n independent-ish steps and a count c independent of z: the second-order term of
    # the mean of a ratio.  It is 0.3% here, above the 0.1% statistical error of the mean.
    return 1.0 + float(np.var(z) / np.mean(z) ** 2)


def test_townsend_paper_form_approaches_rate_over_drift(light_target_run):
    # G_n counts Binomial(n, 0.15) ionisations over the drift length z_n = W t_n + O(sqrt t),
    # t_n = n/nu on average: <G_n/z_n> -> 0.15 nu / W, <D_n/z_n> -> 0.05 nu / W.  W is the
    # run's own drift velocity (with a light target the forward-biased energy loss makes it
    # exceed eE/(m nu) by 1.5%; the W estimator is pinned on the Maxwell gas).
    rec, T = light_target_run
    W = T["W"][0]
    z = -rec["r"][:, 2]
    assert T["n_finished"] == len(rec) and np.all(z > 0)
    bias = _ratio_mean_bias(z)
    _within(T["alpha"][0], 0.15 * NU / W * bias, T["alpha"][1])
    _within(T["eta"][0], 0.05 * NU / W * bias, T["eta"][1])
    # the paper form and the ratio of sums agree to the same second-order term
    assert abs(T["alpha"][0] / T["alpha_rate"] / bias - 1) < 4 * T["alpha"][1] / T["alpha"][0]
    # both are positive along the drift direction (electrons drift against E)
    assert T["alpha"][0] > 0 and T["eta"][0] > 0


def test_townsend_paper_form_spread(light_target_run):
    # The per-electron spread (the printed "+-") of G_n/z_n: G_n is binomial with relative
    # variance (1-p)/(n p) and z_n has the measured relative variance, independent to first
    # order, so spread/mean = sqrt((1-p)/(n p) + Var z / E[z]^2).
    rec, T = light_target_run
    z = -rec["r"][:, 2]
    cz2 = float(np.var(z) / np.mean(z) ** 2)
    n = 4000
    for key, p in (("alpha", 0.15), ("eta", 0.05)):
        want = math.sqrt((1 - p) / (n * p) + cz2)
        assert abs(T[key][2] / T[key][0] / want - 1) < 0.06, (key, T[key][2] / T[key][0], want)


def test_townsend_paper_form_uses_the_finished_set():
    # Real secondaries: an attached electron is removed, so it never finishes.  Over the
    # finished set F every D_n is 0 and <eta> vanishes exactly, although the run attached
    # many electrons (whose D_n = 1 would make an all-electron average positive).  <alpha>
    # over F counts each finished electron's own ionisations.
    comp = synth.constant_rate_component(4.0, 1.0, 0.985 * K, 0.01 * K, 0.005 * K)
    rec = oracle.OracleModel([comp], synth.td_to_field(30.0), secondaries=1).run(2000, 200, 5).records
    T = tallies(rec)
    fin = (rec["flags"] & oracle.FLAG_FINISHED) != 0
    assert T["n_attached"] > 100 and T["n_finished"] == int(fin.sum()) < len(rec)
    assert T["eta"][0] == 0.0 and T["eta"][2] == 0.0 and T["eta_rate"] == 0.0
    assert np.all(rec["D"][fin] == 0) and np.all(rec["D"][~fin] == 1)
    assert T["alpha"][0] > 0


# ---- displacement family: paper form and vector form ----------------------------------

def _records(r, t):
    rec = np.zeros(len(t), dtype=oracle.RECORD_DTYPE)
    rec["id"] = np.arange(len(t))
    rec["flags"] = oracle.FLAG_FINISHED
    rec["k_end"] = 10
    rec["r"] = r
    rec["t"] = t
    return rec


def test_vector_form_removes_a_uniform_drift_exactly():
    # Electrons at r_n = t_n V + rho_n, with the rho_n in +- pairs of equal t (so that the
    # mean of rho_n/t_n is exactly 0): the vector-form drift is V and its displacements are
    # the rho_n, so D_vec, D_L,vec, D_T,vec and sigma_vec are those of the rho_n alone,
    # whatever V is.  The paper form subtracts only V_z t_n along z and keeps the transverse
    # drift: d_n = rho_n + t_n (V_x, V_y, 0), so its D and D_T grow by t_n |V_perp|^2 per
    # electron on average (the +- pairs cancel the cross terms), and its D_L is unchanged.
    rng = np.random.default_rng(3)
    m = 500
    t = np.repeat(rng.uniform(1e-9, 3e-9, m), 2)
    rho = rng.normal(0.0, 2e-5, (m, 3))
    rho = np.stack([rho, -rho], axis=1).reshape(2 * m, 3)
    V = np.array([3.0e3, -4.0e3, -5.0e4])
    T = tallies(_records(t[:, None] * V + rho, t))
    # the rho_n alone, carried by the longitudinal drift only (both forms remove it exactly)
    T0 = tallies(_records(t[:, None] * np.array([0.0, 0.0, V[2]]) + rho, t))
    for key, want in (("Wx", V[0]), ("Wy", V[1]), ("Wz", V[2])):
        assert abs(T[key][0] - want) <= 1e-9 * abs(want), key
    for key in ("D", "DL", "DT", "sigma", "sigmaL", "sigmaT"):
        assert abs(T[key + "_vec"][0] / T0[key][0] - 1) < 1e-9, key
    vp2 = V[0] ** 2 + V[1] ** 2
    assert abs(T["DL"][0] / T0["DL"][0] - 1) < 1e-9
    assert abs(T["sigmaL"][0] / T0["sigmaL"][0] - 1) < 1e-9
    assert abs((T["D"][0] - T0["D"][0]) / (vp2 * t.mean()) - 1) < 1e-9
    assert abs((T["DT"][0] - T0["DT"][0]) / (vp2 * t.mean() / 4) - 1) < 1e-9
    # with no transverse drift both forms coincide
    for key in ("D", "DL", "DT", "sigma", "sigmaL", "sigmaT"):
        assert abs(T0[key][0] / T0[key + "_vec"][0] - 1) < 1e-9, key


def _helix_walk(n, nw, B_T, angle, seed):
    # An independent model of the same process: speed v0 constant (infinitely heavy target,
    # no field E), isotropic directions, exponential flight times of rate NU, and between
    # collisions a helix about b = B/|B|: the velocity component along b is constant, the
    # transverse one, written as a complex number w in the plane (e1, e2) normal to b,
    # turns as w exp(i omega tau) and moves the electron by w (exp(i omega tau) - 1)/(i omega).
    # The sense of rotation does not change the spread.  Returns displacements in the frame
    # z along E, B in the xz plane at `angle` from z, and the times.
    rng = np.random.default_rng(seed)
    v0 = math.sqrt(2 * QE / ME)           # 1 eV
    om = QE * B_T / ME
    dpar = np.zeros(nw)
    dperp = np.zeros(nw, dtype=complex)
    t = np.zeros(nw)
    for _ in range(n):
        cz = rng.uniform(-1.0, 1.0, nw)
        ph = rng.uniform(0.0, 2 * math.pi, nw)
        w = v0 * np.sqrt(1.0 - cz * cz) * np.exp(1j * ph)
        tau = rng.exponential(1.0 / NU, nw)
        dpar += v0 * cz * tau
        dperp += w * np.expm1(1j * om * tau) / (1j * om)
        t += tau
    b = np.array([math.sin(angle), 0.0, math.cos(angle)])
    e1 = np.array([math.cos(angle), 0.0, -math.sin(angle)])
    e2 = np.array([0.0, 1.0, 0.0])
    d = dpar[:, None] * b + dperp.real[:, None] * e1 + dperp.imag[:, None] * e2
    return d, t, dpar, dperp


@pytest.mark.parametrize("angle", [0.0, math.pi / 3])
def test_diffusion_along_and_across_B_against_helix_walk(angle):
    # E = 0, constant rate NU, no energy loss, B with omega = NU (5.69 T).  Along B the
    # motion is that of the field-free walk, D_par = v0^2/(3 NU); across B the gyration cuts
    # the free path: D_perp = v0^2 NU/(3 (NU^2 + omega^2)) = D_par/2 here.  The oracle's
    # paper-form and vector-form D_L, D_T (z along E, B at `angle`) must equal the same
    # estimators on the numpy walk; the walk itself meets the closed forms (with the
    # finite-n factor n/(n+1) of the field-free case along B).
    B = NU * ME / QE
    comp = synth.constant_rate_component(1e9, 1.0, K)
    n, ne = 200, 40000
    T = tallies(oracle.OracleModel([comp], 0.0, B_T=B, B_angle_rad=angle, init_energy_eV=1.0)
                .run(ne, n, 5).records)
    d, t, dpar, dperp = _helix_walk(n, 200_000, B, angle, seed=7)
    walk = {"DL": d[:, 2] ** 2 / (2 * t), "DT": (d[:, 0] ** 2 + d[:, 1] ** 2) / (4 * t),
            "D": (d ** 2).sum(axis=1) / t}
    for key, x in walk.items():
        sw = x.std() / math.sqrt(len(x))
        for form in ("", "_vec"):
            _within(T[key + form][0], x.mean(), math.hypot(T[key + form][1], sw))
    v0sq = 2 * QE / ME
    d_par = v0sq / (3 * NU) * n / (n + 1)
    d_perp = v0sq * NU / (3 * (NU ** 2 + (QE * B / ME) ** 2))
    assert abs(np.mean(dpar ** 2 / (2 * t)) / d_par - 1) < 0.01
    assert abs(np.mean(np.abs(dperp) ** 2 / (4 * t)) / d_perp - 1) < 0.01
    if angle == 0.0:
        # B along E: D_L is the parallel coefficient, D_T the perpendicular one
        assert abs(T["DL"][0] / d_par - 1) < 0.03
        assert abs(T["DT"][0] / d_perp - 1) < 0.03
