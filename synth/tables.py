"""Synthetic cross-section tables (raw points only; no interpolation or rates here).

Every table is a list of (energy [eV], cross-section [m^2]) points with strictly
increasing energies, plus a channel kind and a threshold energy.  The kinds follow
the paper's classes of processes (section "Theoretical framework"): elastic
(momentum-transfer table used with isotropic scattering), excitation, ionisation
and attachment.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ELASTIC, EXCITATION, IONIZATION, ATTACHMENT = 0, 1, 2, 3
KIND_NAMES = {ELASTIC: "elastic", EXCITATION: "excitation", IONIZATION: "ionization",
              ATTACHMENT: "attachment"}


@dataclass
class Channel:
    kind: int
    threshold_eV: float
    energy_eV: np.ndarray
    sigma_m2: np.ndarray
    name: str = ""

    def __post_init__(self):
        self.energy_eV = np.ascontiguousarray(self.energy_eV, dtype=np.float64)
        self.sigma_m2 = np.ascontiguousarray(self.sigma_m2, dtype=np.float64)


@dataclass
class Component:
    mass_amu: float
    fraction: float
    channels: list = field(default_factory=list)
    name: str = ""
    scattering: int = 0          # 0 isotropic, 1 screened Coulomb (atomic), 2 constant xi (molecular)
    mt_over_el: float = 1.0      # scattering 2: sigma_mt / sigma_el, in (0, 1]

    def with_fraction(self, fraction: float) -> "Component":
        return Component(self.mass_amu, float(fraction), list(self.channels), self.name, self.scattering,
                         self.mt_over_el)

    def with_scattering(self, scattering: int, mt_over_el: float = 1.0) -> "Component":
        return Component(self.mass_amu, self.fraction, list(self.channels), self.name, int(scattering),
                         float(mt_over_el))


def grid_node_energies(points_per_octave: int = 64, min_exp2: int = -14, max_exp2: int = 12):
    """Energies 2^e * (1 + i/P) for every octave e in [min_exp2, max_exp2) and i < P,
    followed by 2^max_exp2.  A table sampled exactly here is reproduced without
    interpolation error on an octave grid with the same parameters."""
    out = []
    for e in range(min_exp2, max_exp2):
        base = math.ldexp(1.0, e)
        for i in range(points_per_octave):
            out.append(base * (1.0 + i / points_per_octave))
    out.append(math.ldexp(1.0, max_exp2))
    return np.array(out, dtype=np.float64)


# ---------------------------------------------------------------------------
# Maxwell-model gas: sigma = k / sqrt(eps) makes nu = N k sqrt(2e/m_e) constant.
# k = 6.744260e-20 m^2 eV^0.5 gives nu = 1.000e12 s^-1 at N = 2.5e25 m^-3.
# ---------------------------------------------------------------------------
MAXWELL_K = 6.744260e-20


def maxwell_component(mass_amu: float = 4.0, fraction: float = 1.0, k: float = MAXWELL_K,
                      points_per_octave: int = 64, min_exp2: int = -14, max_exp2: int = 12):
    e = grid_node_energies(points_per_octave, min_exp2, max_exp2)
    s = k / np.sqrt(e)
    return Component(mass_amu, fraction, [Channel(ELASTIC, 0.0, e, s, "maxwell-elastic")],
                     f"maxwell-{mass_amu:g}u")


def constant_rate_component(mass_amu: float, fraction: float, k_el: float, k_ion: float = 0.0,
                            k_att: float = 0.0, points_per_octave: int = 64,
                            min_exp2: int = -14, max_exp2: int = 12):
    """Channels whose cross-sections all scale as 1/sqrt(eps), with zero thresholds,
    so that each channel has an energy-independent rate.  Used for closed-form checks
    of the ionisation and attachment bookkeeping."""
    e = grid_node_energies(points_per_octave, min_exp2, max_exp2)
    rs = 1.0 / np.sqrt(e)
    ch = [Channel(ELASTIC, 0.0, e, k_el * rs, "const-elastic")]
    if k_ion > 0:
        ch.append(Channel(IONIZATION, 0.0, e, k_ion * rs, "const-ionization"))
    if k_att > 0:
        ch.append(Channel(ATTACHMENT, 0.0, e, k_att * rs, "const-attachment"))
    return Component(mass_amu, fraction, ch, f"const-{mass_amu:g}u")


def _rise_decay(eps, eps_k, eps_p, sigma_p):
    """Linear rise from the threshold to a peak, then (eps_p/eps) ln(eps/eps_k) decay."""
    eps = np.asarray(eps, dtype=np.float64)
    out = np.zeros_like(eps)
    rise = (eps > eps_k) & (eps <= eps_p)
    out[rise] = sigma_p * (eps[rise] - eps_k) / (eps_p - eps_k)
    tail = eps > eps_p
    out[tail] = sigma_p * (eps_p / eps[tail]) * np.log(eps[tail] / eps_k) / math.log(eps_p / eps_k)
    return out


def _inelastic_points(eps_k, eps_p, e_max=1000.0, n=100):
    pts = np.geomspace(eps_k, e_max, n)
    pts = np.unique(np.concatenate([pts, [eps_p]]))
    return pts


def _ramsauer_elastic(eps, eps_min=0.23, scale=1.0):
    x = np.log(eps / eps_min)
    return scale * 1e-20 * (0.1 + 12.0 * x * x / (x * x + 4.0)) / (1.0 + (eps / 20.0) ** 0.8)


def argon_like(mass_amu: float = 40.0, fraction: float = 1.0):
    """Argon-like atom: Ramsauer minimum near 0.23 eV, three excitations
    (11.5, 11.8, 13.0 eV) and ionisation at 15.8 eV."""
    e_el = np.geomspace(0.01, 1000.0, 200)
    ch = [Channel(ELASTIC, 0.0, e_el, _ramsauer_elastic(e_el), "ar-elastic")]
    for eps_k, sp in zip((11.5, 11.8, 13.0), (1.0e-21, 0.5e-21, 2.0e-21)):
        eps_p = eps_k + 4.0
        e = _inelastic_points(eps_k, eps_p)
        ch.append(Channel(EXCITATION, eps_k, e, _rise_decay(e, eps_k, eps_p, sp), f"ar-exc-{eps_k:g}"))
    e = _inelastic_points(15.8, 80.0)
    ch.append(Channel(IONIZATION, 15.8, e, _rise_decay(e, 15.8, 80.0, 2.5e-20), "ar-ion"))
    return Component(mass_amu, fraction, ch, f"argon-like-{mass_amu:g}u")


def co2_like(fraction: float = 1.0):
    """CO2-like molecule (44 u): 13 vibrational excitations (0.08-1.0 eV), 7 electronic
    excitations (7-11 eV), dissociative attachment peaked at 8 eV, ionisation at 13.8 eV."""
    e_el = np.geomspace(0.01, 1000.0, 200)
    s_el = 1e-20 * (1.2 / np.sqrt(e_el + 0.01) + 10.0 * e_el / ((e_el + 5.0) * (1.0 + e_el / 30.0)))
    ch = [Channel(ELASTIC, 0.0, e_el, s_el, "co2-elastic")]
    vib_sp = np.geomspace(3e-21, 2e-22, 13)
    for i in range(13):
        eps_k = 0.08 * 12.5 ** (i / 12.0)
        eps_p = 1.5 * eps_k + 0.05
        e = _inelastic_points(eps_k, eps_p)
        ch.append(Channel(EXCITATION, eps_k, e, _rise_decay(e, eps_k, eps_p, vib_sp[i]), f"co2-vib-{i}"))
    ele_sp = np.geomspace(5e-22, 2e-21, 7)
    for i in range(7):
        eps_k = 7.0 + 4.0 * i / 6.0
        eps_p = eps_k + 5.0
        e = _inelastic_points(eps_k, eps_p)
        ch.append(Channel(EXCITATION, eps_k, e, _rise_decay(e, eps_k, eps_p, ele_sp[i]), f"co2-el-{i}"))
    e_da = np.linspace(4.0, 12.0, 100)
    s_da = 4e-23 * np.exp(-(e_da - 8.0) ** 2 / (2 * 0.8 ** 2))
    ch.append(Channel(ATTACHMENT, 0.0, e_da, s_da, "co2-da"))
    e = _inelastic_points(13.8, 90.0)
    ch.append(Channel(IONIZATION, 13.8, e, _rise_decay(e, 13.8, 90.0, 3.5e-20), "co2-ion"))
    return Component(44.0, fraction, ch, "co2-like")


def random_component(rng: np.random.Generator, fraction: float = 1.0, max_inelastic: int = 24):
    """A random molecule: mass 2-200 u, a Ramsauer-shaped elastic table with a random
    minimum and scale, 0..max_inelastic inelastic channels (excitations, at most one
    ionisation, at most one attachment) and 100-400 table points per channel."""
    mass = 10 ** rng.uniform(math.log10(2.0), math.log10(200.0))
    n_pts = int(rng.integers(100, 401))
    e_el = np.geomspace(0.01, 1000.0, n_pts)
    eps_min = 10 ** rng.uniform(-1.0, 0.0)
    scale = 10 ** rng.uniform(-0.5, 0.5)
    ch = [Channel(ELASTIC, 0.0, e_el, _ramsauer_elastic(e_el, eps_min, scale), "rnd-elastic")]
    n_inel = int(rng.integers(0, max_inelastic + 1))
    have_ion = have_att = False
    for _ in range(n_inel):
        r = rng.uniform()
        n_pts = int(rng.integers(100, 401))
        if r < 0.1 and not have_ion:
            have_ion = True
            eps_k = rng.uniform(10.0, 25.0)
            eps_p = eps_k * rng.uniform(3.0, 8.0)
            e = _inelastic_points(eps_k, eps_p, n=n_pts)
            sp = 10 ** rng.uniform(math.log10(5e-21), math.log10(5e-20))
            ch.append(Channel(IONIZATION, eps_k, e, _rise_decay(e, eps_k, eps_p, sp), "rnd-ion"))
        elif r < 0.2 and not have_att:
            have_att = True
            peak = rng.uniform(1.0, 10.0)
            width = rng.uniform(0.3, 1.5)
            e = np.linspace(max(peak - 5 * width, 0.01), peak + 5 * width, n_pts)
            sp = 10 ** rng.uniform(-24.0, -21.0)
            ch.append(Channel(ATTACHMENT, 0.0, e, sp * np.exp(-(e - peak) ** 2 / (2 * width * width)),
                              "rnd-att"))
        else:
            eps_k = 10 ** rng.uniform(math.log10(0.05), math.log10(20.0))
            eps_p = eps_k * rng.uniform(1.2, 3.0) + 0.05
            e = _inelastic_points(eps_k, eps_p, n=n_pts)
            sp = 10 ** rng.uniform(-22.0, -20.0)
            ch.append(Channel(EXCITATION, eps_k, e, _rise_decay(e, eps_k, eps_p, sp), "rnd-exc"))
    return Component(mass, fraction, ch, f"random-{mass:.1f}u")
