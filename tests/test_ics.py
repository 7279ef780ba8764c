"""Pins for the synthetic input generators against numbers the paper prints
(tests/golden/paper_values.json, each with its citation) and closed forms."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1507_01009_amd import ics

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_hernquist_half_mass_radius():
    g = GOLD["hernquist_half_mass_radius"]
    assert ics.dehnen_half_mass_radius(1.0) == pytest.approx(1 + math.sqrt(2), rel=1e-14)
    assert abs(ics.dehnen_half_mass_radius(1.0) - g["value"]) < g["tol"]


@pytest.mark.parametrize("key", ["hernquist_vcirc_at_half_mass", "hernquist_vcirc_at_0.1"])
def test_hernquist_circular_speeds(key):
    g = GOLD[key]
    assert abs(float(ics.dehnen_vcirc(g["r"], 1.0)) - g["value"]) < g["tol"]


def test_unit_conversions():
    G = 6.674e-11
    msun, kpc, myr = 1.989e30, 3.0857e19, 3.15576e13
    M, L = GOLD["time_unit_myr"]["mass_msun"] * msun, GOLD["time_unit_myr"]["length_kpc"] * kpc
    t = math.sqrt(L ** 3 / (G * M)) / myr
    v = math.sqrt(G * M / L) / 1e3
    assert abs(t - GOLD["time_unit_myr"]["value"]) < GOLD["time_unit_myr"]["tol"]
    assert abs(v - GOLD["velocity_unit_kms"]["value"]) < GOLD["velocity_unit_kms"]["tol"]


def test_eddington_df_matches_hernquist_closed_form():
    df = ics.EddingtonDF(1.0)
    E = np.array([1e-3, 0.01, 0.1, 0.3, 0.5, 0.7, 0.9, 0.99])
    assert np.allclose(df(E), ics.hernquist_df_exact(E), rtol=2e-4)


def test_dehnen_radii_follow_enclosed_mass():
    pos, _, _ = ics.dehnen(20000, 1.5, 4)
    r = np.sort(np.linalg.norm(pos, axis=1))
    for q in (0.1, 0.3, 0.5, 0.8):
        rq = r[int(q * r.size)]
        assert float(ics.dehnen_mass(rq, 1.5)) / 0.99 == pytest.approx(q, abs=0.02)


@pytest.mark.parametrize("gamma", [0.5, 1.0, 1.5])
def test_dehnen_virial_equilibrium(gamma):
    pos, vel, m = ics.dehnen(8192, gamma, 40 + int(2 * gamma))
    _, pot = oracle.direct(pos, m, 1e-3)
    K = 0.5 * np.sum(m * np.sum(vel * vel, 1))
    W = 0.5 * np.sum(m * pot)
    assert 2 * K / abs(W) == pytest.approx(1.0, abs=0.06)


def test_plummer_virial_and_radii():
    pos, vel, m = ics.plummer(8192, 3)
    r = np.sort(np.linalg.norm(pos, axis=1))
    rh = r[r.size // 2]
    assert rh == pytest.approx(1.0 / math.sqrt(2 ** (2 / 3) - 1), rel=0.05)
    _, pot = oracle.direct(pos, m, 1e-3)
    K = 0.5 * np.sum(m * np.sum(vel * vel, 1))
    W = 0.5 * np.sum(m * pot)
    assert 2 * K / abs(W) == pytest.approx(1.0, abs=0.05)


def test_binary_setup_circular_speed():
    w = ics.cusp_c3(n=4096)
    r = 0.005
    v = math.sqrt(r * (0.005 / 0.01 ** 2 + float(ics.dehnen_mass(r, 1.5)) / r ** 2))
    assert np.allclose(np.abs(w.bh_vel[:, 1]), v)
    assert np.allclose(w.bh_pos[:, 0], [r, -r])


def test_generators_are_seeded():
    a = ics.dehnen(1000, 1.0, 5)
    b = ics.dehnen(1000, 1.0, 5)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    c = ics.batch_c5(S=4, nmin=1000, nmax=3000)
    assert c.sys_off.shape == (5,) and c.pos.shape[0] == c.sys_off[-1]
