"""Pins of the energy-transfer formulas (Fraser-Mathieson, the paper's eqs. delta_energy_ela
and delta_energy_ine) against exact two-body kinematics computed with vectors."""
import math

import numpy as np
import pytest

import oracle

QE, ME, AMU = oracle.constants()
ELA, EXC, ION, ATT = 0, 1, 2, 3


def exact_two_body(eps, eps_k, cos_chi, M):
    """Electron energy after a collision with a target at rest that absorbs eps_k of
    internal energy, for centre-of-momentum scattering angle chi: momentum and energy
    conservation written out with vectors."""
    m = ME
    v = np.array([0.0, 0.0, math.sqrt(2 * eps * QE / m)])
    V = m * v / (m + M)                      # centre-of-momentum velocity
    g = np.linalg.norm(v)                    # relative speed (target at rest)
    mu = m * M / (m + M)
    e_rel = 0.5 * mu * g * g - eps_k * QE    # relative kinetic energy after the loss
    g2 = math.sqrt(2 * e_rel / mu)
    sin_chi = math.sqrt(max(0.0, 1 - cos_chi ** 2))
    ghat = np.array([sin_chi, 0.0, cos_chi])
    v_after = V + (M / (m + M)) * g2 * ghat
    return 0.5 * m * v_after @ v_after / QE


@pytest.mark.parametrize("M_amu", [4.0, 40.0, 44.0, 1.0])
def test_elastic_formula_is_exact_kinematics(M_amu):
    rng = np.random.default_rng(3)
    for _ in range(200):
        eps = 10 ** rng.uniform(-3, 3)
        c = rng.uniform(-1, 1)
        got = oracle.energy_after(ELA, eps, 0.0, c, M_amu)
        want = exact_two_body(eps, 0.0, c, M_amu * AMU)
        assert abs(got - want) <= 1e-12 * eps


@pytest.mark.parametrize("M_amu", [4.0, 40.0, 44.0, 1.0])
def test_inelastic_formula_is_exact_kinematics(M_amu):
    rng = np.random.default_rng(4)
    M = M_amu * AMU
    for _ in range(300):
        eps_k = 10 ** rng.uniform(-2, 1.3)
        onset = eps_k * (ME + M) / M
        eps = onset * (1 + 10 ** rng.uniform(-8, 2))
        c = rng.uniform(-1, 1)
        got = oracle.energy_after(EXC, eps, eps_k, c, M_amu)
        want = exact_two_body(eps, eps_k, c, M)
        assert abs(got - want) <= 1e-9 * eps
        assert got >= -1e-12 * eps          # allowed collisions leave non-negative energy
        assert oracle.energy_after(ION, eps, eps_k, c, M_amu) == got


def test_zero_threshold_reduces_to_elastic():
    for c in np.linspace(-1, 1, 21):
        for eps in (0.01, 1.0, 300.0):
            a = oracle.energy_after(EXC, eps, 0.0, c, 40.0)
            b = oracle.energy_after(ELA, eps, 0.0, c, 40.0)
            assert abs(a - b) <= 1e-15 * eps


def test_attachment_is_plastic():
    assert oracle.energy_after(ATT, 7.0, 0.0, 0.3, 44.0) == 0.0


def test_mean_elastic_loss_fraction():
    # averaged over isotropic cos(theta) the energy kept is 1 - 2mM/(m+M)^2
    M = 4.0 * AMU
    cs = np.linspace(-1, 1, 2001)
    kept = np.mean([oracle.energy_after(ELA, 1.0, 0.0, c, 4.0) for c in cs])
    assert abs(kept - (1 - 2 * ME * M / (ME + M) ** 2)) < 1e-12
