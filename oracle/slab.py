"""FP64 reference of the planar long-range correction of the LJ force.

TEST INFRASTRUCTURE ONLY: used by the test suite, never by the product
package; it shares no code with the GPU path.

The slab runs of Sec. 5.2 add a long-range correction to the two-body forces
and cite it without stating it.  This module writes it out from the LJ pair
force for a laterally uniform density: a sheet of areal density s_a at height
offset xi = z_i - z' exerts on molecule i the z-force of all its molecules
farther than rc,

    F_z = s_a * integral over r >= max(rc, |xi|) of f(r) (xi / r) 2 pi r dr
        = 2 pi s_a xi phi(max(rc, |xi|)),

with phi(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] and f = -phi' (the lateral
integral of f xi / r over r from R to infinity is xi (phi(R) - 0)).  The
density profile is binned: bin k of nbins over L_z (centre (k + 1/2) L_z /
nbins) carries s_a = n_k / (L_x L_y), and xi is the minimum image in z.
Every molecule of bin b receives the force evaluated at b's centre, so the
pair of bins (b, k) contributes opposite forces n_b n_k (...) and the
correction adds no net momentum.
"""
from __future__ import annotations

import math

import numpy as np


def z_bins(pos, box, nbins):
    """Bin of each molecule: z <- z - L_z floor(z / L_z), k = floor(z * (nbins / L_z))
    clamped to [0, nbins - 1] (FP64, the same expression as the library's)."""
    lz = float(box[2])
    z = np.asarray(pos, dtype=np.float64)[:, 2]
    z = z - lz * np.floor(z / lz)
    k = np.floor(z * (float(nbins) / lz)).astype(np.int64)
    return np.clip(k, 0, nbins - 1)


def z_histogram(pos, box, nbins):
    """Molecules per z bin."""
    return np.bincount(z_bins(pos, box, nbins), minlength=nbins).astype(np.int64)


def sheet_force(xi, areal, rc, eps=1.0, sigma=1.0):
    """z-force on a molecule at offset xi from a uniform sheet of areal
    density `areal`, from the sheet's molecules beyond rc (closed form above)."""
    xi = np.asarray(xi, dtype=np.float64)
    r = np.maximum(rc, np.abs(xi))
    s6 = (sigma / r) ** 6
    return 2.0 * math.pi * areal * xi * 4.0 * eps * (s6 * s6 - s6)


def bin_forces(hist, box, rc, eps=1.0, sigma=1.0):
    """Correction z-force at each bin centre from the binned profile."""
    lx, ly, lz = (float(b) for b in box)
    nbins = len(hist)
    centres = (np.arange(nbins) + 0.5) * (lz / nbins)
    xi = centres[:, None] - centres[None, :]
    xi = xi - lz * np.rint(xi / lz)
    return sheet_force(xi, np.asarray(hist, dtype=np.float64)[None, :] / (lx * ly), rc, eps, sigma).sum(axis=1)


def lrc_forces(pos, box, nbins, rc, eps=1.0, sigma=1.0):
    """z-component of the long-range correction on every molecule (the force
    at its bin's centre) and the histogram it is built from."""
    k = z_bins(pos, box, nbins)
    hist = np.bincount(k, minlength=nbins).astype(np.int64)
    return bin_forces(hist, box, rc, eps, sigma)[k], hist
