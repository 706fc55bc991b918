"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only builds inputs: raw cross-section tables (energy in eV, cross-section
in m^2), gas-mixture descriptions and run configurations.  It contains none of the
swarm method's arithmetic (no interpolation, no rates, no motion, no tallies), so the
oracle and the HIP path can both consume it without sharing any method code.

The paper (Betaboltz, arXiv 1901.08140) measures on LXCat tables, which are not
available here; the shapes below stand in for them (argon-like with a Ramsauer
minimum, CO2-like with vibrational and electronic excitations, dissociative
attachment and ionisation, a Maxwell-model gas, and random components).
"""
from .tables import (  # noqa: F401
    Channel, Component, ELASTIC, EXCITATION, IONIZATION, ATTACHMENT,
    maxwell_component, argon_like, co2_like, random_component, constant_rate_component,
    grid_node_energies,
)
from .configs import (  # noqa: F401
    SwarmConfig, td_to_field, cfg1_maxwell, cfg2_argon_sweep, cfg2_td_values, cfg3_mixture_real,
    cfg4_batch, cfg4_mixtures, cfg5_request, cfg5_requests, mixture_ar_co2, N_DEFAULT, DUMMY, REAL,
)
