"""The paper's table of jet conditions (tests/golden/jet_table.txt, Results: the table of
simulation data) against the parameter arithmetic of the jet setups, Re = U D / nu and
We = rho U^2 D / sigma with rho = 1 (Results, opening paragraph)."""
import os

import numpy as np
import pytest

from paper_2403_15773_amd import inputs

ROWS = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "jet_table.txt"))


def test_table_shape_and_domain():
    assert ROWS.shape == (5, 10)
    for r in ROWS:
        D, nx, ny, nz = r[4], r[5], r[6], r[7]
        # the domain of 10 D x 10 D x 20 D, 128 million nodes (caption of the domain figure)
        assert (nx, ny, nz) == (10 * D, 10 * D, 20 * D) and nx * ny * nz == 128e6


@pytest.mark.parametrize("row", [3, 4])  # sims 4 and 5
def test_jet_setup_reproduces_the_consistent_rows(row):
    sim, U, sigma, nu, D, nx, ny, nz, Re, We = ROWS[row]
    p = inputs.jet_params(int(nx), int(ny), int(nz), d=D, u=U, re=Re, we=We)
    assert p["nu"] == pytest.approx(nu, rel=1e-12)
    assert p["sigma"] == pytest.approx(sigma, rel=1e-12)
    assert p["inlet_u"] == U and p["inlet_d"] == D


def test_rows_1_to_3_do_not_follow_from_their_parameters():
    """Reading of the table: the printed Re and We of sims 1-3 are not those of their printed
    U, sigma and nu (Re 5970 and 6395, We 10, 89 and 143), so the jet setups derive nu and
    sigma from Re and We and never take rows 1-3 as parameter sets."""
    U, sigma, nu, D, Re, We = ROWS[:3, 1], ROWS[:3, 2], ROWS[:3, 3], ROWS[:3, 4], ROWS[:3, 8], ROWS[:3, 9]
    re_implied, we_implied = U * D / nu, U * U * D / sigma
    assert np.allclose(re_implied, [5970.1, 6395.2, 6395.2], rtol=1e-3)
    assert np.allclose(we_implied, [10.0, 89.1, 142.6], rtol=1e-3)
    assert np.all(np.abs(re_implied / Re - 1) > 0.15)
    assert np.abs(we_implied[1:] / We[1:] - 1).min() > 0.4


def test_every_row_keeps_the_mach_number_low():
    """Ma = U / c_s with c_s = 1/sqrt(3) stays well below 0.6 (Results, before the table)."""
    assert np.all(ROWS[:, 1] * np.sqrt(3.0) < 0.6)
