"""Helpers shared by the GPU parity tests (comparison of records, events and tallies)."""
import math

import numpy as np

INT_FIELDS = ["id", "flags", "k_start", "k_end", "G", "D", "n_forbidden", "n_over", "n_fail", "n_null",
              "blocks"]
FLOAT_FIELDS = ["t", "sum_eps", "sum_epsp"]


def sort_by_id(rec):
    return rec[np.argsort(rec["id"], kind="stable")]


def compare_records(gpu, ora, rtol=1e-9):
    """Element-by-element comparison: integer fields exact, continuous fields to rtol."""
    g = sort_by_id(gpu)
    o = sort_by_id(ora)
    assert len(g) == len(o), (len(g), len(o))
    for f in INT_FIELDS:
        bad = np.nonzero(g[f] != o[f])[0]
        assert len(bad) == 0, f"field {f}: {len(bad)} mismatches, first id {o['id'][bad[0]]}: gpu {g[f][bad[0]]} oracle {o[f][bad[0]]}"
    for f in FLOAT_FIELDS:
        a, b = g[f], o[f]
        err = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
        assert np.all((err <= rtol) | (a == b)), f"field {f}: max rel err {err.max():.3e}"
    # positions: relative to the largest displacement component scale of the electron
    scale = np.maximum(np.max(np.abs(o["r"]), axis=1), 1e-30)
    err = np.max(np.abs(g["r"] - o["r"]), axis=1) / scale
    assert np.all(err <= rtol), f"positions: max rel err {err.max():.3e}"


def compare_events(gev, gcount, oev, ids, rtol=1e-9):
    for i, eid in enumerate(ids):
        oe = oev[oev["id"] == eid]
        ge = gev[i, :gcount[i]]
        assert len(ge) == len(oe), (eid, len(ge), len(oe))
        for f in ("type", "channel", "k", "block", "sub"):
            assert np.array_equal(ge[f], oe[f]), (eid, f)
        for f in ("eps", "epsp", "t"):
            a, b = ge[f], oe[f]
            err = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
            assert np.all((err <= rtol) | (a == b)), (eid, f, err.max())


PARITY_KEYS = ["W", "Wx", "Wy", "Wz", "mean_energy", "mean_energy_after", "D", "DL", "DT", "sigma",
               "sigmaL", "sigmaT", "D_vec", "DL_vec", "DT_vec", "sigma_vec", "sigmaL_vec", "sigmaT_vec",
               "alpha", "eta"]


def tally_agreement(a, b, keys=PARITY_KEYS, k=3.0, rel=0.005):
    """Statistical agreement of two independent estimates: |dx| <= k sqrt(sa^2+sb^2) + rel |x_b|.
    Returns the list of (key, a, b, allowed) that fail."""
    bad = []
    for key in keys:
        va, sa, _ = a[key]
        vb, sb, _ = b[key]
        if not (math.isfinite(va) and math.isfinite(vb)):
            if not (math.isnan(va) and math.isnan(vb)):
                bad.append((key, va, vb, float("nan")))
            continue
        allowed = k * math.hypot(sa, sb) + rel * abs(vb)
        if abs(va - vb) > allowed:
            bad.append((key, va, vb, allowed))
    return bad


PAIRED_KEYS = ["W", "mean_energy", "mean_energy_after", "D", "DL", "DT", "alpha"]


def per_electron(rec):
    """Per-electron contributions to the mean-type tallies of the finished electrons (dummy
    mode: every electron makes the same number of collisions, so the mean energies are means
    of sum/k too), each with its own run's drift velocity in the displacement."""
    fin = (rec["flags"] & 1) != 0
    rec = rec[fin]
    r, t = rec["r"], rec["t"]
    k = (rec["k_end"].astype(np.int64) - rec["k_start"]).astype(float)
    wz = np.mean(r[:, 2] / t)
    dz = r[:, 2] - t * wz
    dp2 = r[:, 0] ** 2 + r[:, 1] ** 2
    return rec["id"], {"W": -r[:, 2] / t, "mean_energy": rec["sum_eps"] / k, "mean_energy_after": rec["sum_epsp"] / k,
                       "D": (dz ** 2 + dp2) / t, "DL": dz ** 2 / (2 * t), "DT": dp2 / (4 * t),
                       "alpha": rec["G"] / -r[:, 2]}


def paired_bias(rec_a, rec_b, keys=PAIRED_KEYS):
    """Bias of run a against run b on the same electrons (same ids, same random streams):
    {key: (mean_a - mean_b, its standard error from the per-electron paired differences,
    mean_b)}.  Runs that share streams are strongly correlated, so the paired error is far
    below that of two independent estimates."""
    a, b = sort_by_id(rec_a), sort_by_id(rec_b)
    ida, qa = per_electron(a)
    idb, qb = per_electron(b)
    assert np.array_equal(ida, idb), "the runs finished different electrons"
    out = {}
    for key in keys:
        d = qa[key] - qb[key]
        out[key] = (float(np.mean(d)), float(np.std(d, ddof=1) / math.sqrt(len(d))), float(np.mean(qb[key])))
    return out


def paired_bias_failures(pb, k=4.0, floor=2e-5):
    """Keys whose bias exceeds k paired standard errors plus floor x |value|."""
    return [(key, bias, sig, ref) for key, (bias, sig, ref) in pb.items()
            if not abs(bias) <= k * sig + floor * abs(ref)]
