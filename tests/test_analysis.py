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
