"""Pins of the oracle's lattices and single-node collision operators.

The checks are moment identities the paper's construction fixes (Methodology:
Eqs. 2, 5, 7, 15-19 for the hydrodynamics; Eqs. 23-24 for the phase field),
computed by summing the oracle's populations numerically.  A dropped term, a
wrong sign or index, or c c in place of the Hermite H2 fails one of them.
"""
import itertools

import numpy as np
import pytest

from oracle import collide, lattice, phase_collide

CS2 = 1.0 / 3.0
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


@pytest.fixture(scope="module")
def lat(oracle_lib):
    return lattice()


def _sym(P):
    m = np.zeros((3, 3))
    for s, (a, b) in enumerate(PAIRS):
        m[a, b] = m[b, a] = P[s]
    return m


def _cases(n=20, seed=0):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        rho = 1.0 + 0.2 * rng.uniform(-1, 1)
        u = 0.1 * rng.uniform(-1, 1, 3)
        P = 0.01 * rng.uniform(-1, 1, 6)
        F = 0.01 * rng.uniform(-1, 1, 3)
        omega = rng.uniform(0.5, 1.99)
        yield rho, u, P, F, omega


def test_d3q27_velocity_set_and_weights(lat):
    c, w, _, _ = lat
    assert len({tuple(v) for v in c}) == 27
    for i in range(27):
        assert tuple(c[i]) == (i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1)
    # three speed groups |c| = 1, sqrt 2, sqrt 3 plus rest (D3Q27 figure)
    s = (c * c).sum(1)
    assert sorted(np.bincount(s)) == sorted([1, 6, 12, 8])
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    # isotropy through fourth order: sum w c_a c_b = cs2 d_ab,
    # sum w c_a c_b c_g c_d = cs2^2 (d_ab d_gd + d_ag d_bd + d_ad d_bg), odd moments vanish
    I = np.eye(3)
    m2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(m2, CS2 * I, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ig,id->abgd", w, c, c, c, c)
    iso4 = CS2 ** 2 * (np.einsum("ab,gd->abgd", I, I) + np.einsum("ag,bd->abgd", I, I)
                       + np.einsum("ad,bg->abgd", I, I))
    assert np.allclose(m4, iso4, atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ig->abg", w, c, c, c), 0, atol=1e-16)
    # tensor-product structure of the D3Q27 weights: sixth moment cs2^3
    assert np.einsum("i,i,i,i->", w, c[:, 0] ** 2, c[:, 1] ** 2, c[:, 2] ** 2) == pytest.approx(CS2 ** 3)


def test_d3q7_velocity_set(lat):
    _, _, c7, w7 = lat
    assert w7.sum() == pytest.approx(1.0)
    assert np.allclose(np.einsum("k,ka,kb->ab", w7, c7, c7), 0.25 * np.eye(3))
    assert np.allclose(np.einsum("k,ka->a", w7, c7), 0)


@pytest.mark.parametrize("case", list(_cases()))
def test_hydro_moments_through_second_order(lat, case):
    c, _, _, _ = lat
    rho, u, P, F, omega = case
    f = collide(rho, u, P, F, omega)
    # mass: sum f^post = rho (every correction has zero zeroth moment)
    assert f.sum() == pytest.approx(rho, abs=1e-14)
    # momentum: sum f^post c = rho u + F/2 = j + F  (Guo, u = (j + F/2)/rho)
    assert np.allclose(c.T @ f, rho * u + 0.5 * F, atol=1e-15)
    # momentum flux: rho cs2 I + rho u u + (1 - omega) P + (u F + F u)/2
    M2 = np.einsum("i,ia,ib->ab", f, c, c)
    exp = rho * CS2 * np.eye(3) + rho * np.outer(u, u) + (1 - omega) * _sym(P) + 0.5 * (np.outer(u, F) + np.outer(F, u))
    assert np.allclose(M2, exp, atol=1e-15)


@pytest.mark.parametrize("case", list(_cases(seed=1)))
def test_hydro_third_order_moments(lat, case):
    """Eq. 17 (equilibrium third moment) and Eqs. 18-19 (regularised third order)."""
    c, _, _, _ = lat
    rho, u, P, F, omega = case
    Pm = _sym(P)
    f = collide(rho, u, P, F, omega)
    x, y, z = 0, 1, 2
    # xyz: a^3_xyz = rho u_x u_y u_z + (1 - omega)(u_x P_yz + u_y P_xz + u_z P_xy)
    m_xyz = (f * c[:, x] * c[:, y] * c[:, z]).sum()
    assert m_xyz == pytest.approx(rho * u[x] * u[y] * u[z]
                                  + (1 - omega) * (u[x] * Pm[y, z] + u[y] * Pm[x, z] + u[z] * Pm[x, y]), abs=1e-15)
    # aab (a != b): cs2 (rho u_b + F_b/2) + rho u_a^2 u_b + (1 - omega)(2 u_a P_ab + u_b P_aa)
    for a, b in itertools.permutations(range(3), 2):
        m = (f * c[:, a] ** 2 * c[:, b]).sum()
        exp = CS2 * (rho * u[b] + 0.5 * F[b]) + rho * u[a] ** 2 * u[b] + (1 - omega) * (2 * u[a] * Pm[a, b] + u[b] * Pm[a, a])
        assert m == pytest.approx(exp, abs=1e-15)


@pytest.mark.parametrize("case", list(_cases(n=6, seed=2)))
def test_equilibrium_third_moment_eq17(lat, case):
    """Eq. 17: Q_abb = sum f^eq c_a c_b c_b, here with P = 0, F = 0 so f^post = f^eq:
    Q_xyy = rho (u_x u_y^2 + cs2 u_x); Q_xxx = rho u_x (lattice degeneracy c^3 = c)."""
    c, _, _, _ = lat
    rho, u, _, _, omega = case
    f = collide(rho, u, np.zeros(6), np.zeros(3), omega)
    for a in range(3):
        for b in range(3):
            q = (f * c[:, a] * c[:, b] ** 2).sum()
            exp = rho * u[a] if a == b else rho * (u[a] * u[b] ** 2 + CS2 * u[a])
            assert q == pytest.approx(exp, abs=1e-15)


@pytest.mark.parametrize("case", list(_cases(n=6, seed=3)))
def test_no_hermite_content_above_third_order(lat, case):
    """Eqs. 16 and 19 stop at n = 3: every Hermite moment of order 4..6 vanishes."""
    c, _, _, _ = lat
    rho, u, P, F, omega = case
    f = collide(rho, u, P, F, omega)
    h1 = c.astype(float)
    h2 = c * c - CS2
    for a, b in itertools.combinations(range(3), 2):
        assert abs((f * h2[:, a] * h2[:, b]).sum()) < 1e-15
    for a in range(3):
        b, g = [k for k in range(3) if k != a]
        assert abs((f * h2[:, a] * h1[:, b] * h1[:, g]).sum()) < 1e-15
        assert abs((f * h2[:, b] * h2[:, g] * h1[:, a]).sum()) < 1e-15
    assert abs((f * h2[:, 0] * h2[:, 1] * h2[:, 2]).sum()) < 1e-15


def test_equilibrium_reduces_to_eq2_at_low_mach(lat):
    """Eq. 16 differs from the second-order Maxwellian of Eq. 2 only at O(u^3)."""
    c, w, _, _ = lat
    rng = np.random.default_rng(5)
    u0 = rng.uniform(-1, 1, 3)
    diffs = []
    for scale in (0.04, 0.02, 0.01):
        u = scale * u0
        f = collide(1.0, u, np.zeros(6), np.zeros(3), 1.0)
        cu = c @ u
        feq2 = w * (1 + cu / CS2 + (cu * cu - CS2 * (u @ u)) / (2 * CS2 ** 2))
        diffs.append(np.abs(f - feq2).max())
    assert diffs[0] / diffs[1] == pytest.approx(8.0, rel=1e-6)
    assert diffs[1] / diffs[2] == pytest.approx(8.0, rel=1e-6)


def test_unit_relaxation_erases_nonequilibrium(lat):
    rng = np.random.default_rng(6)
    u = 0.05 * rng.uniform(-1, 1, 3)
    F = 1e-3 * rng.uniform(-1, 1, 3)
    a = collide(1.1, u, 0.01 * rng.uniform(-1, 1, 6), F, 1.0)
    b = collide(1.1, u, np.zeros(6), F, 1.0)
    assert np.allclose(a, b, atol=1e-17)


@pytest.mark.parametrize("seed", range(8))
def test_phase_moments(lat, seed):
    """Eqs. 23-24: sum g = phi; sum g c = phi u + cs_phi^2 gamma phi (1-phi) n; sum g c c = cs_phi^2 phi I."""
    _, _, c7, _ = lat
    rng = np.random.default_rng(100 + seed)
    phi = rng.uniform(0, 1)
    u = 0.1 * rng.uniform(-1, 1, 3)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    gamma = rng.uniform(0.1, 1.0)
    g = phase_collide(phi, u, n, gamma)
    assert g.sum() == pytest.approx(phi, abs=1e-15)
    assert np.allclose(c7.T @ g, phi * u + 0.25 * gamma * phi * (1 - phi) * n, atol=1e-15)
    assert np.allclose(np.einsum("k,ka,kb->ab", g, c7, c7), 0.25 * phi * np.eye(3), atol=1e-15)
