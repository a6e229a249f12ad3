"""CPU checks of the jet-statistics post-processing on synthetic mean fields
whose decay constant, virtual origin and half-width are known."""
import numpy as np
import pytest

from paper_2403_15773_amd import analysis


def _synthetic_jet(nx=65, ny=65, nz=200, U=0.05, D=8.0, B=6.0, z0=-2.0, spread=0.1):
    """Self-similar round jet: U_c(z) = U B D / (z - z0 D), Gaussian radial profile
    with half-width b(z) = spread (z - z0 D) (exp(-ln2 r^2 / b^2))."""
    z = np.arange(nz, dtype=np.float64)
    uc = U * B * D / (z - z0 * D)
    b = spread * (z - z0 * D)
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - (nx - 1) / 2.0) ** 2 + (y - (ny - 1) / 2.0) ** 2
    f = uc[:, None, None] * np.exp(-np.log(2.0) * r2[None] / b[:, None, None] ** 2)
    return f, uc, b


def test_centreline_and_decay_constant():
    f, uc, _ = _synthetic_jet()
    line = analysis.centreline(f)
    assert np.allclose(line, uc, rtol=1e-12)  # odd width: the axis is a node
    # an even width puts the axis between nodes; the bilinear value is exact for a plane
    ramp = np.broadcast_to(np.arange(8.0)[None, None, :] + 2 * np.arange(8.0)[None, :, None], (3, 8, 8))
    assert np.allclose(analysis.centreline(ramp), 3.5 + 7.0)
    B, z0 = analysis.decay_constant(uc, 0.05, 8.0, (40, 200))
    assert B == pytest.approx(6.0, rel=1e-9) and z0 == pytest.approx(-2.0, abs=1e-9)


def test_half_width_of_a_gaussian_profile():
    f, _, b = _synthetic_jet()
    for z in (60, 120, 180):
        assert analysis.half_width(f[z]) == pytest.approx(b[z], rel=0.03)


def test_radial_profile_of_a_constant_is_constant():
    r, prof = analysis.radial_profile(np.full((32, 32), 3.0))
    assert np.allclose(prof, 3.0) and r[0] == 0.5


def test_gaussian_exponent_of_a_self_similar_profile():
    """b = spread (z - z0 D) with exp(-ln2 r^2 / b^2) is exp(-K eta^2) with
    K = ln2 / spread^2 and eta = r / (z - z0 D)."""
    f, _, _ = _synthetic_jet(nx=129, ny=129, nz=200, spread=0.1)
    K = np.log(2.0) / 0.1 ** 2
    for z in (80, 150):
        assert analysis.gaussian_exponent(f[z], z, -16.0) == pytest.approx(K, rel=0.02)
    # the slope of 1/phi_c: phi_c = B D / (z - z0 D) with U = 1
    _, uc, _ = _synthetic_jet(U=1.0, B=6.5, z0=0.6)  # origin off the grid: 4.8
    B, z0 = analysis.decay_constant(uc, 1.0, 8.0, (30, 200))
    assert B == pytest.approx(6.5, rel=1e-9) and z0 == pytest.approx(0.6, abs=1e-9)


def test_jetstats_rejects_an_empty_averaging_window():
    from paper_2403_15773_amd import jetstats
    with pytest.raises(SystemExit):
        jetstats.main(["--steps", "100", "--avg-from", "100"])
