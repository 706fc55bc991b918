"""Swarm tallies from per-electron records, with the paper's estimators (section
"Determination of swarm attributes").  TEST INFRASTRUCTURE ONLY (plain numpy, FP64).

Frame: z along E; electrons (charge -e) drift towards -z, so the scalar drift velocity and
the Townsend coefficients are taken along h = -z (the printed worked example reports a
positive W).  The completed set F holds the electrons that made all their real collisions.

Each tally is returned as (value, stat_sigma, spread): `spread` is the sample standard
deviation of the per-electron quantity (the paper's printed "+-"), `stat_sigma` = spread /
sqrt(N_F), the statistical uncertainty of the mean.

Pins (tests/test_oracle_swarm.py, tests/test_oracle_estimators.py): W against eE/(m nu) and
the Drude drift; the mean energies against their closed form; D, D_L, D_T field-free and
along/across B against closed forms and an independent helical random walk; sigma, sigma_L,
sigma_T against a random walk; the vector form's removal of a uniform drift, exactly, on
hand-built records; alpha, eta (per-electron and ratio-of-sums forms) against constant rates.
"""
from __future__ import annotations

import numpy as np

from . import FLAG_ATTACHED, FLAG_FINISHED, FLAG_STUCK


def _mean_stats(x):
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n == 0:
        return (float("nan"), float("nan"), float("nan"))
    m = float(np.mean(x))
    s = float(np.std(x, ddof=1)) if n > 1 else 0.0
    return (m, s / np.sqrt(n), s)


def tallies(records):
    rec = records
    fin = (rec["flags"] & FLAG_FINISHED) != 0
    F = rec[fin]
    out = {}
    k_real = (rec["k_end"].astype(np.int64) - rec["k_start"].astype(np.int64))
    K_real = int(k_real.sum())
    K_null = int(rec["n_null"].astype(np.int64).sum())
    K_forb = int(rec["n_forbidden"].astype(np.int64).sum())
    out["n_real"] = K_real
    out["n_null"] = K_null
    out["n_forbidden"] = K_forb
    K_fail = int(rec["n_fail"].astype(np.int64).sum())
    out["n_fail"] = K_fail
    out["n_over"] = int(rec["n_over"].astype(np.int64).sum())
    out["n_electrons"] = int(len(rec))
    out["n_finished"] = int(fin.sum())
    out["n_attached"] = int(((rec["flags"] & FLAG_ATTACHED) != 0).sum())
    out["n_stuck"] = int(((rec["flags"] & FLAG_STUCK) != 0).sum())
    out["n_created"] = int((rec["id"] >> np.uint64(63) != 0).sum())
    out["n_ionizations"] = int(rec["G"].astype(np.int64).sum())
    out["n_attachments"] = int(rec["D"].astype(np.int64).sum())
    trials = K_real + K_null + K_forb + K_fail
    # Efficiency (section "Trial frequency strategies"): real / (real + null + fail);
    # forbidden events count as null trials.
    out["efficiency"] = K_real / trials if trials else float("nan")

    # Mean energies before and after the collisions: plain means over every real collision.
    if K_real:
        out["mean_energy"] = float(rec["sum_eps"].sum()) / K_real
        out["mean_energy_after"] = float(rec["sum_epsp"].sum()) / K_real
        has = k_real > 0
        per_e = rec["sum_eps"][has] / k_real[has]
        per_ep = rec["sum_epsp"][has] / k_real[has]
        _, se, sd = _mean_stats(per_e)
        _, sep, sdp = _mean_stats(per_ep)
        out["mean_energy"] = (out["mean_energy"], se, sd)
        out["mean_energy_after"] = (out["mean_energy_after"], sep, sdp)
    else:
        out["mean_energy"] = out["mean_energy_after"] = (float("nan"),) * 3

    r = F["r"]
    t = F["t"]
    # Drift velocity W = (1/N) sum z_n / t_n, as a vector and along h = -z.
    vx, vy, vz = r[:, 0] / t, r[:, 1] / t, r[:, 2] / t
    Wx, Wy, Wz = _mean_stats(vx), _mean_stats(vy), _mean_stats(vz)
    out["Wx"], out["Wy"], out["Wz"] = Wx, Wy, Wz
    out["W"] = (-Wz[0], Wz[1], Wz[2])

    # Displacement from the mean drift, d_n = x_n - t_n W z^ (paper form, W = z-component).
    d = r.copy()
    d[:, 2] = r[:, 2] - t * Wz[0]
    _diffusion(out, d, t, "")
    # Vector form: d_n = x_n - t_n W_vec (removes the E x B drift as well).
    dv = r - t[:, None] * np.array([Wx[0], Wy[0], Wz[0]])[None, :]
    _diffusion(out, dv, t, "_vec")

    # Townsend coefficients with dummy/real counts G_n, D_n over z_n (along h).
    zh = -r[:, 2]
    out["alpha"] = _mean_stats(F["G"] / zh)
    out["eta"] = _mean_stats(F["D"] / zh)
    szh = float(zh.sum())
    out["alpha_rate"] = float(F["G"].astype(np.float64).sum()) / szh if len(F) else float("nan")
    out["eta_rate"] = float(F["D"].astype(np.float64).sum()) / szh if len(F) else float("nan")
    return out


def _diffusion(out, d, t, suffix):
    dz2 = d[:, 2] ** 2
    dp2 = d[:, 0] ** 2 + d[:, 1] ** 2
    out["D" + suffix] = _mean_stats((dz2 + dp2) / t)
    out["DL" + suffix] = _mean_stats(dz2 / (2.0 * t))
    out["DT" + suffix] = _mean_stats(dp2 / (4.0 * t))
    out["sigma" + suffix] = _mean_stats(2.0 * np.sqrt(dz2 + dp2))
    out["sigmaL" + suffix] = _mean_stats(2.0 * np.abs(d[:, 2]))
    out["sigmaT" + suffix] = _mean_stats(2.0 * np.sqrt(dp2))


TALLY_KEYS = ["W", "Wx", "Wy", "Wz", "mean_energy", "mean_energy_after", "D", "DL", "DT",
              "sigma", "sigmaL", "sigmaT", "D_vec", "DL_vec", "DT_vec", "sigma_vec",
              "sigmaL_vec", "sigmaT_vec", "alpha", "eta"]
