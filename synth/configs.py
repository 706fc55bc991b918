"""Run configurations (the five workloads) built from the synthetic tables.

Field values are given as reduced fields E/N in townsend (1 Td = 1e-21 V m^2);
`td_to_field` turns them into V/m for the gas density N.  The geometry is the paper's
swarm set-up (section "Determination of swarm attributes"): z along E, B in the xz
plane at an angle to E.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from .tables import Component, argon_like, co2_like, maxwell_component, random_component

N_DEFAULT = 2.5e25      # m^-3
T_DEFAULT = 293.0       # K (bookkeeping: the targets are at rest)
EPS0_DEFAULT = 0.1      # eV, initial electron energy
DUMMY, REAL = 0, 1


def td_to_field(e_over_n_td: float, n_per_m3: float = N_DEFAULT) -> float:
    return e_over_n_td * 1e-21 * n_per_m3


@dataclass
class SwarmConfig:
    components: list
    E_V_per_m: float
    B_T: float = 0.0
    B_angle_rad: float = 0.0
    N_per_m3: float = N_DEFAULT
    T_K: float = T_DEFAULT
    init_energy_eV: float = EPS0_DEFAULT
    secondaries: int = DUMMY
    n_electrons: int = 1000
    n_collisions: int = 1000
    seed: int = 0
    user_majorant: float = 0.0
    trial_strategy: int = 0      # 0 constant trial frequency, 1 variable (zeta, grace),
                                 # 2 binned (bins per decade, grace)
    trial_zeta: float = 0.25
    trial_grace: int = 5000
    trial_bins: int = 10
    thermal_targets: int = 0     # 1: targets with Maxwell-Boltzmann velocities at T_K
    relativistic: int = 0        # 1: relativistic motion (B = 0)
    label: str = ""
    extra: dict = field(default_factory=dict)

    def scaled(self, n_electrons=None, n_collisions=None, **kw):
        c = replace(self, **kw)
        if n_electrons is not None:
            c.n_electrons = int(n_electrons)
        if n_collisions is not None:
            c.n_collisions = int(n_collisions)
        return c


def cfg1_maxwell(n_electrons=1000, n_collisions=10_000, seed=0):
    """Maxwell-model gas, M = 4 u, nu = 1e12 s^-1, E/N = 10 Td, B = 0, DUMMY mode."""
    return SwarmConfig([maxwell_component(4.0)], td_to_field(10.0), n_electrons=n_electrons,
                       n_collisions=n_collisions, seed=seed, label="maxwell-10Td")


def cfg2_td_values():
    return [10 ** (3.0 * i / 31.0) for i in range(32)]


def cfg2_argon_sweep(n_electrons=100_000, n_collisions=20_000, seed=0):
    """Argon-like gas at 32 log-spaced E/N from 1 to 1000 Td, B = 0, DUMMY mode."""
    comp = [argon_like()]
    return [SwarmConfig(comp, td_to_field(td), n_electrons=n_electrons, n_collisions=n_collisions,
                        seed=seed, label=f"argon-{td:.4g}Td", extra={"td": td})
            for td in cfg2_td_values()]


def mixture_ar_co2(ar=0.9, co2=0.1):
    return [argon_like(fraction=ar), co2_like(fraction=co2)]


def cfg3_mixture_real(n_electrons=1_000_000, n_collisions=50_000, seed=0):
    """90:10 argon-like:CO2-like at 100 Td with B = 1 T at 45 degrees, REAL secondaries."""
    return SwarmConfig(mixture_ar_co2(), td_to_field(100.0), B_T=1.0, B_angle_rad=math.pi / 4,
                       secondaries=REAL, n_electrons=n_electrons, n_collisions=n_collisions,
                       seed=seed, label="arco2-100Td-1T45")


def cfg4_mixtures():
    m1 = [argon_like()]
    m2 = mixture_ar_co2()
    m3 = [argon_like(fraction=0.8), co2_like(fraction=0.1), maxwell_component(4.0, fraction=0.1)]
    m4 = [argon_like(fraction=0.7), co2_like(fraction=0.1), maxwell_component(4.0, fraction=0.1),
          argon_like(mass_amu=84.0, fraction=0.1)]
    return [m1, m2, m3, m4]


def cfg4_batch(seed=4):
    """256 instances: 4 mixtures x 64 log-spaced E/N over 1-1000 Td; B is 0 or 1 T
    (probability 1/2) at an angle uniform in [0, pi); electron counts log-uniform in
    1e3-1e6 and collision budgets log-uniform in 1e3-1e5.  Run seed = instance index."""
    rng = np.random.default_rng(seed)
    mixes = cfg4_mixtures()
    tds = np.geomspace(1.0, 1000.0, 64)
    out = []
    idx = 0
    for mi, mix in enumerate(mixes):
        for td in tds:
            has_b = rng.uniform() < 0.5
            ang = rng.uniform(0.0, math.pi)
            ne = int(round(10 ** rng.uniform(3.0, 6.0)))
            nc = int(round(10 ** rng.uniform(3.0, 5.0)))
            out.append(SwarmConfig(mix, td_to_field(float(td)), B_T=1.0 if has_b else 0.0,
                                   B_angle_rad=ang if has_b else 0.0, n_electrons=ne,
                                   n_collisions=nc, seed=idx,
                                   label=f"m{mi + 1}-{td:.4g}Td", extra={"td": float(td), "mix": mi}))
            idx += 1
    return out


def cfg5_request(i: int, base_seed: int = 5, max_components: int = 6):
    """Request i of the serving stream: 1..max_components random components with
    Dirichlet(1) fractions, E/N log-uniform in 1-1000 Td, |B| uniform in 0-2 T at an angle
    uniform in [0, pi), electrons log-uniform in 1e3-1e6, collisions in 1e3-1e5."""
    rng = np.random.default_rng([base_seed, i])
    nc_comp = int(rng.integers(1, max_components + 1))
    fr = rng.dirichlet(np.ones(nc_comp))
    comps = [random_component(rng, fraction=float(f)) for f in fr]
    s = sum(c.fraction for c in comps)
    for c in comps:
        c.fraction /= s
    td = 10 ** rng.uniform(0.0, 3.0)
    b = rng.uniform(0.0, 2.0)
    ang = rng.uniform(0.0, math.pi)
    ne = int(round(10 ** rng.uniform(3.0, 6.0)))
    nc = int(round(10 ** rng.uniform(3.0, 5.0)))
    return SwarmConfig(comps, td_to_field(td), B_T=b, B_angle_rad=ang, n_electrons=ne,
                       n_collisions=nc, seed=i, label=f"req-{i}", extra={"td": td})


def cfg5_requests(rate_per_s=50.0, duration_s=600.0, seed=5):
    """Poisson arrival times of the serving stream (the requests themselves come from
    `cfg5_request`)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    times = []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        times.append(t)
    return np.array(times)
