"""Jet statistics from time-averaged fields (host-side post-processing).

The averages come from the device (``Simulation.stats()``); this module only
reads them (Results, self-similarity of the jets):
* the centreline values along the jet axis;
* the linear law of an inverse centreline value, ref / X_c(z) = (z - z0) / (B D)
  beyond the potential core, for the axial velocity (ref = U) and for the phase
  field (ref = 1); the paper reports a slope 1/B of about 1/6.5 per diameter;
* the Gaussian exponent K of a radial profile X / X_c = exp(-K eta^2) with
  eta = r / (z - z0) (the paper compares K = 80 for the phase field and K = 75
  for the axial velocity with experiments);
* the half-width b(z) where a profile falls to half its centreline value.
"""
from __future__ import annotations

import numpy as np


def centreline(field, axis_x=None, axis_y=None):
    """Values of field (nz, ny, nx) on the line through (axis_x, axis_y), by
    bilinear interpolation; the default axis is ((nx-1)/2, (ny-1)/2)."""
    nz, ny, nx = field.shape
    ax = (nx - 1) / 2.0 if axis_x is None else axis_x
    ay = (ny - 1) / 2.0 if axis_y is None else axis_y
    i0, j0 = int(np.floor(ax)), int(np.floor(ay))
    fx, fy = ax - i0, ay - j0
    i1, j1 = min(i0 + 1, nx - 1), min(j0 + 1, ny - 1)
    f = np.asarray(field, np.float64)
    return ((1 - fx) * (1 - fy) * f[:, j0, i0] + fx * (1 - fy) * f[:, j0, i1] +
            (1 - fx) * fy * f[:, j1, i0] + fx * fy * f[:, j1, i1])


def decay_constant(uc, U, D, z_window):
    """Fit U/U_c(z) = (z - z0)/(B D) on z in [z_window[0], z_window[1]) (plane
    indices); returns (B, z0/D).  With U = 1 and the centreline phase field it
    gives the slope of 1/phi_c."""
    z = np.arange(len(uc), dtype=np.float64)
    sel = (z >= z_window[0]) & (z < z_window[1])
    slope, icept = np.polyfit(z[sel] / D, U / np.asarray(uc, np.float64)[sel], 1)
    return 1.0 / slope, -icept / slope


def radial_profile(plane, nbins=None, axis_x=None, axis_y=None):
    """Azimuthal average of a (ny, nx) plane around the axis: (r, mean) with
    unit-width bins in r."""
    ny, nx = plane.shape
    ax = (nx - 1) / 2.0 if axis_x is None else axis_x
    ay = (ny - 1) / 2.0 if axis_y is None else axis_y
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - ax) ** 2 + (y - ay) ** 2)
    nb = int(min(ax, ay)) if nbins is None else nbins
    k = np.floor(r).astype(int)
    sums = np.bincount(k.ravel(), weights=np.asarray(plane, np.float64).ravel(), minlength=nb + 1)[:nb]
    counts = np.bincount(k.ravel(), minlength=nb + 1)[:nb]
    with np.errstate(invalid="ignore"):
        return np.arange(nb) + 0.5, sums / np.maximum(counts, 1)


def half_width(plane, axis_x=None, axis_y=None):
    """Radius where the azimuthally averaged value first drops to half of the
    centreline value (linear interpolation between bins)."""
    r, prof = radial_profile(plane, axis_x=axis_x, axis_y=axis_y)
    c = centreline(np.asarray(plane)[None], axis_x, axis_y)[0]
    below = np.nonzero(prof < 0.5 * c)[0]
    if len(below) == 0 or below[0] == 0:
        return float("nan")
    k = below[0]
    return float(r[k - 1] + (0.5 * c - prof[k - 1]) * (r[k] - r[k - 1]) / (prof[k] - prof[k - 1]))


def gaussian_exponent(plane, z, z0, cutoff=0.05, axis_x=None, axis_y=None):
    """Least-squares K of ln(X/X_c) = -K eta^2, eta = r / (z - z0), over the
    radial bins with X/X_c above `cutoff` (plane = the (ny, nx) slice at z;
    z and z0 in lattice units)."""
    r, prof = radial_profile(plane, axis_x=axis_x, axis_y=axis_y)
    c = centreline(np.asarray(plane)[None], axis_x, axis_y)[0]
    y = prof / c
    sel = np.isfinite(y) & (y > cutoff) & (y < 1.0)
    eta2 = (r[sel] / (z - z0)) ** 2
    return float(-np.sum(eta2 * np.log(y[sel])) / np.sum(eta2 * eta2))
