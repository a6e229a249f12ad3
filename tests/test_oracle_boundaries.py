"""Pins of the oracle's boundary layers (Eqs. 9-10: equilibrium from imposed
rho and/or u, non-equilibrium taken from the nearest interior node x_F).

The jet's boundary rules have no closed-form solution to compare against, so
beyond these rule checks the jet path is "parity unpinned" against physics:
only oracle-versus-GPU comparisons cover it.
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle.oracle import BC_FREESLIP as FS, BC_INLET as IN, BC_OUTFLOW as OUT, BC_NOSLIP as NS
from paper_2403_15773_amd import inputs

PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def _random_state(nx, ny, nz, seed):
    sh = (nz, ny, nx)
    node = np.arange(nx * ny * nz, dtype=np.uint64)
    nz_ = lambda s, c: inputs.noise(seed, s, 0, node, c).reshape(sh)  # noqa: E731
    return {"rho": 1.0 + 0.01 * nz_(0, 0), "u": 0.02 * np.stack([nz_(1, a) for a in range(3)]),
            "P": 1e-3 * np.stack([nz_(2, a) for a in range(6)]), "phi": 0.5 + 0.4 * nz_(3, 0)}


@pytest.fixture(scope="module")
def jet(oracle_lib):
    nx, ny, nz = 10, 12, 14
    U, D, W, a, seed = 0.05, 6.0, 3.0, 0.01, 4
    o = Oracle(nx, ny, nz, nu=0.01, sigma=0.001, width=W, bc=(FS, FS, FS, FS, IN, OUT),
               inlet_u=U, inlet_d=D, inlet_noise=a, seed=seed)
    o.set_physical(**_random_state(nx, ny, nz, 21), step=37)
    raw = o.raw()
    return dict(o=o, raw=raw, nx=nx, ny=ny, nz=nz, U=U, D=D, W=W, a=a, seed=seed)


def _xf(v, n):
    return min(max(v, 1), n - 2)


def test_inlet_imposes_velocity_and_phase(jet):
    r, nx, ny = jet["raw"], jet["nx"], jet["ny"]
    for y in range(ny):
        for x in range(nx):
            rr = np.hypot(x - (nx - 1) / 2, y - (ny - 1) / 2)
            s = 0.5 * (1 - np.tanh(2 * (rr - jet["D"] / 2) / jet["W"]))
            xi = inputs.noise(jet["seed"], 1, 37, x + nx * y, 2)
            assert r["ubar"][2][0, y, x] == pytest.approx(jet["U"] * s * (1 + jet["a"] * xi), abs=2e-15)
            assert abs(r["ubar"][0][0, y, x]) < 1e-15 and abs(r["ubar"][1][0, y, x]) < 1e-15
            assert r["phi"][0, y, x] == pytest.approx(s, abs=2e-15)
            xf, yf = _xf(x, nx), _xf(y, ny)
            assert r["drho"][0, y, x] == pytest.approx(r["drho"][1, yf, xf], abs=1e-15)
            assert np.allclose(r["Q"][:, 0, y, x], r["Q"][:, 1, yf, xf], atol=2e-15)


def test_outflow_fixes_density_and_copies_the_rest(jet):
    r, nx, ny, nz = jet["raw"], jet["nx"], jet["ny"], jet["nz"]
    top = nz - 1
    for y in range(ny):
        for x in range(nx):
            xf, yf = _xf(x, nx), _xf(y, ny)
            assert r["drho"][top, y, x] == pytest.approx(0.0, abs=1e-15)
            assert np.allclose(r["ubar"][:, top, y, x], r["ubar"][:, top - 1, yf, xf], atol=2e-15)
            assert np.allclose(r["Q"][:, top, y, x], r["Q"][:, top - 1, yf, xf], atol=2e-15)
            assert r["phi"][top, y, x] == pytest.approx(r["phi"][top - 1, yf, xf], abs=1e-15)


@pytest.mark.parametrize("axis", [0, 1])
def test_free_slip_walls(jet, axis):
    """Normal velocity and normal-tangential stress vanish; the rest is copied.
    Edges shared with a z face follow the z face; x-y edges follow the y face."""
    r, nx, ny, nz = jet["raw"], jet["nx"], jet["ny"], jet["nz"]
    for z in range(1, nz - 1):
        for y in range(ny):
            for x in range(nx):
                on_y = y in (0, ny - 1)
                on_x = x in (0, nx - 1)
                face = 1 if on_y else 0 if on_x else None
                if face != axis:
                    continue
                xf, yf = _xf(x, nx), _xf(y, ny)
                assert abs(r["ubar"][axis][z, y, x]) < 1e-15
                for a in range(3):
                    if a != axis:
                        assert r["ubar"][a][z, y, x] == pytest.approx(r["ubar"][a][z, yf, xf], abs=2e-15)
                for s, (a, b) in enumerate(PAIRS):
                    if (a == axis) != (b == axis):
                        assert abs(r["Q"][s][z, y, x]) < 1e-15
                    else:
                        assert r["Q"][s][z, y, x] == pytest.approx(r["Q"][s][z, yf, xf], abs=2e-15)
                assert r["phi"][z, y, x] == pytest.approx(r["phi"][z, yf, xf], abs=1e-15)


def test_no_slip_wall(oracle_lib):
    nx, ny, nz = 6, 6, 6
    o = Oracle(nx, ny, nz, nu=0.05, sigma=0.0, bc=(0, 0, 0, 0, NS, NS))
    o.set_physical(**_random_state(nx, ny, nz, 22))
    r = o.raw()
    assert np.abs(r["ubar"][:, 0]).max() < 1e-15 and np.abs(r["ubar"][:, -1]).max() < 1e-15
    assert np.allclose(r["Q"][:, 0], r["Q"][:, 1], atol=2e-15)


def test_mini_jet_runs_and_injects_phase(oracle_lib):
    """A 16x16x24 jet (D = 6) for 150 steps stays finite and fills with phase."""
    p = inputs.jet_params(16, 16, 24, d=6.0, u=0.05, re=300.0, we=50.0, seed=5)
    o = Oracle(16, 16, 24, nu=p["nu"], sigma=p["sigma"], width=p["width"], bc=p["bc"], inlet_u=p["inlet_u"],
               inlet_d=p["inlet_d"], inlet_noise=p["inlet_noise"], seed=p["seed"], eps=1e-4)
    o.set_physical(**inputs.quiescent(16, 16, 24))
    _, ph0 = o.sums()
    o.step(150)
    ph = o.physical()
    _, ph1 = o.sums()
    assert all(np.isfinite(v).all() for v in ph.values())
    assert ph1 > ph0 + 10.0
    assert ph["u"][2][1:6, 8, 8].min() > 0.02  # the jet core moves downstream
    assert np.abs(ph["u"]).max() < 0.2


def test_invalid_parameters_are_rejected(oracle_lib):
    with pytest.raises(ValueError):
        Oracle(8, 8, 8, nu=0.0)
    with pytest.raises(ValueError):
        Oracle(8, 8, 8, nu=0.1, bc=(FS, 0, 0, 0, 0, 0))  # periodic pairs must match
    with pytest.raises(ValueError):
        Oracle(8, 8, 8, nu=0.1, bc=(IN, FS, 0, 0, 0, 0))  # inlet only on -z
