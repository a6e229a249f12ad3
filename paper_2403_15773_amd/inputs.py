"""Seeded synthetic inputs shared by the GPU path, its tests and the oracle.

This module holds no arithmetic of the lattice Boltzmann method: it draws
initial fields (a spherical droplet with a tanh profile, velocity noise, a
quiescent jet domain) and describes workloads as plain parameter sets.  The
same arrays are handed to the GPU library and to the oracle.

Noise is a counter-based generator, the SplitMix64 finaliser of
(key XOR counter) with key = SplitMix64(seed) (Steele, Lea and Flood, 2014),
so every value is a pure function of (seed, stream, step, node, component):
  counter = stream * 2**62 + step * 2**32 + node * 4 + comp,
  xi      = (top 24 bits) * 2**-23 - 1  in [-1, 1), exact in float32.
"""
from __future__ import annotations

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)

BC_PERIODIC, BC_FREESLIP, BC_INLET, BC_OUTFLOW, BC_NOSLIP = 0, 1, 2, 3, 4


def _finalise(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def splitmix64_next(state):
    """First SplitMix64 output of ``state``."""
    with np.errstate(over="ignore"):
        return _finalise(np.asarray(state, dtype=np.uint64) + _GOLDEN)


def noise(seed, stream, step, node, comp):
    """Uniform xi in [-1, 1) (float64 holding a float32-exact value)."""
    key = splitmix64_next(np.uint64(seed))
    node = np.asarray(node, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = ((np.uint64(stream) << np.uint64(62)) + (np.uint64(step) << np.uint64(32))
               + (node << np.uint64(2)) + np.uint64(comp))
    h = _finalise(key ^ ctr)
    return (h >> np.uint64(40)).astype(np.float64) * (1.0 / 8388608.0) - 1.0


def grid_coords(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x, y, z


def quiescent(nx, ny, nz, phi=0.0):
    """rho = 1, u = 0, P = 0, phi = const (physical fields, SoA, shape (.., nz, ny, nx))."""
    sh = (nz, ny, nx)
    return {"rho": np.ones(sh), "u": np.zeros((3,) + sh), "P": np.zeros((6,) + sh),
            "phi": np.full(sh, float(phi))}


def droplet(n, radius, width=3.0, noise_amp=1e-3, seed=1, stream=0, center=None, rho_inside=None):
    """Periodic n^3 box with one droplet: phi = (1 - tanh(2 (r - R) / W)) / 2.

    r is the minimum-image distance to ``center`` (default (n/2, n/2, n/2)).
    u_a = noise_amp * xi(seed, stream, step 0, node, a); rho = 1 (or a
    pressure-balanced rho if ``rho_inside`` gives the inside excess rho - 1);
    P = 0.
    """
    if center is None:
        center = (n / 2.0, n / 2.0, n / 2.0)
    x, y, z = grid_coords(n, n, n)
    d = []
    for c, v in zip(center, (x, y, z)):
        dv = v - c
        dv = dv - n * np.round(dv / n)
        d.append(dv)
    r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
    phi = 0.5 * (1.0 - np.tanh(2.0 * (r - radius) / width))
    node = (x + n * (y + n * z)).astype(np.uint64)
    u = np.stack([noise_amp * noise(seed, stream, 0, node, a) for a in range(3)])
    rho = np.ones_like(phi)
    if rho_inside is not None:
        rho = 1.0 + rho_inside * (phi - phi.mean())
    return {"rho": rho, "u": u, "P": np.zeros((6,) + phi.shape), "phi": phi}


def smooth_state(nx, ny, nz):
    """A smooth synthetic state with no quiescent node (binary32, separable
    products of sines): phi in [0.1, 0.9] with interfaces about 10 nodes wide,
    |u| <= 0.02, rho - 1 ~ 1e-3, P ~ 1e-4; keys rho_dev, u, P, phi in the layout
    the library takes; cheap to generate for 5e8 nodes."""
    x, y, z = (np.arange(n, dtype=np.float32) for n in (nx, ny, nz))
    s = lambda v, L, ph=0.0: np.sin(np.float32(2 * np.pi / L) * v + np.float32(ph)).astype(np.float32)  # noqa: E731
    sh = (nz, ny, nx)
    st = {"rho_dev": np.empty(sh, np.float32), "u": np.empty((3,) + sh, np.float32),
          "P": np.empty((6,) + sh, np.float32), "phi": np.empty(sh, np.float32)}
    zy = lambda a, b: (a[:, None] * b[None, :])[:, :, None]  # noqa: E731
    np.multiply(zy(s(z, 41.0), s(y, 29.0)), 0.4 * s(x, 37.0)[None, None, :], out=st["phi"])
    st["phi"] += np.float32(0.5)
    np.multiply(zy(s(z, 17.0), np.ones(ny, np.float32)), 1e-3 * s(x, 53.0, 1.0)[None, None, :], out=st["rho_dev"])
    for a, (Lx, Ly, Lz) in enumerate(((23.0, 31.0, 47.0), (27.0, 19.0, 43.0), (33.0, 25.0, 39.0))):
        np.multiply(zy(s(z, Lz, a), s(y, Ly, 2 * a)), 0.02 * s(x, Lx, 0.5 + a)[None, None, :], out=st["u"][a])
    for k in range(6):
        np.multiply(zy(s(z, 29.0 + k, k), s(y, 23.0 + k)), 1e-4 * s(x, 31.0 + k, 0.3 * k)[None, None, :], out=st["P"][k])
    return st


def taylor_green(n, u0=0.05):
    """Periodic n^3 Taylor-Green vortex: with x_i = 2 pi i / n,
    u = u0 sin x cos y cos z, v = -u0 cos x sin y cos z, w = 0,
    rho = 1 + u0^2 / (16 c_s^2) (cos 2x + cos 2y)(cos 2z + 2), P = 0, phi = 0."""
    k = 2.0 * np.pi / n
    x, y, z = (np.arange(n, dtype=np.float64) * k for _ in range(3))
    X, Y, Z = x[None, None, :], y[None, :, None], z[:, None, None]
    sh = (n, n, n)
    u = np.zeros((3,) + sh)
    u[0] = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    rho = 1.0 + (u0 * u0 / (16.0 / 3.0)) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    return {"rho": np.broadcast_to(rho, sh).copy(), "u": u, "P": np.zeros((6,) + sh), "phi": np.zeros(sh)}


# ---- workloads: plain parameter sets in lattice units ----

def droplet_params(n=32, nu=0.01, sigma=0.01, width=3.0):
    return dict(nx=n, ny=n, nz=n, nu=nu, sigma=sigma, width=width, bc=(BC_PERIODIC,) * 6)


def jet_params(nx, ny, nz, d, u, re, we, width=3.0, noise=0.01, seed=2):
    """Round jet: inlet disc on z = 0, outflow at z = nz-1, free-slip lateral walls.
    Re = U D / nu and We = rho U^2 D / sigma with rho = 1."""
    return dict(nx=nx, ny=ny, nz=nz, nu=u * d / re, sigma=u * u * d / we, width=width,
                bc=(BC_FREESLIP, BC_FREESLIP, BC_FREESLIP, BC_FREESLIP, BC_INLET, BC_OUTFLOW),
                inlet_u=u, inlet_d=d, inlet_noise=noise, seed=seed)


WORKLOADS = {
    # 256^3 periodic Taylor-Green vortex, one component, U0 = 0.05, Re = U0 (n / 2 pi) / nu = 1600
    "tgv256": dict(params=dict(nx=256, ny=256, nz=256, nu=0.05 * (256 / (2 * np.pi)) / 1600.0, sigma=0.0, width=3.0,
                               bc=(BC_PERIODIC,) * 6, components=1), steps=1000, init="taylor_green"),
    # 32^3 periodic droplet, R = 8, W = 3, nu = 0.01, sigma = 0.01, 200 steps
    "droplet32": dict(params=droplet_params(32), steps=200, init="droplet"),
    # 128x128x512 round jet, D = 20, U = 0.05, Re = 5000, We = 100, 2000 steps
    "jet128": dict(params=jet_params(128, 128, 512, d=20, u=0.05, re=5000, we=100, seed=2), steps=2000,
                   init="quiescent"),
    # 512x512x2048 round jet, D = 40, U = 0.05, Re = 5000, We = 2000, 200 warm-up + 500 timed
    "jet512": dict(params=jet_params(512, 512, 2048, d=40, u=0.05, re=5000, we=2000, seed=3), steps=500,
                   init="quiescent"),
    # the paper's own jet domain (Results, Table 1; Performances: 128 million nodes): 400x400x800,
    # D = 40 (10 D x 10 D x 20 D), U = 0.05, Re = 5000, We = 2000
    "jet400": dict(params=jet_params(400, 400, 800, d=40, u=0.05, re=5000, we=2000, seed=4), steps=500,
                   init="quiescent"),
    # the 128x128x512 jet with components of different density: the injected component ten times
    # denser than the ambient, equal viscosities (Re = 5000 in the jet), We = 100
    "jet128vd": dict(params=jet_params(128, 128, 512, d=20, u=0.05, re=5000, we=100, seed=2)
                     | dict(density_a=10.0, density_b=1.0, nu_a=2e-4, nu_b=2e-4), steps=2000, init="quiescent"),
}
