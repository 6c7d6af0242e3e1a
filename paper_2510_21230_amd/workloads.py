"""Seeded synthetic inputs: positions (and velocities) of LJ fluids.

This module holds no part of the force method; it only draws inputs, which the
GPU path and the oracle then both consume.  Workload shapes follow the
paper's own synthetic fluids (Sec. 5: lattice starts, reduced units) and the
benchmark configurations of this package:

* ``fcc``      -- FCC lattice filling a cubic periodic box at density rho,
                  ``n`` of its sites kept by a seeded permutation, each
                  coordinate jittered by U(-jitter, +jitter) sigma;
* ``sc``       -- simple cubic lattice in a cubic box (single-phase start,
                  Sec. 5.1);
* ``uniform``  -- uniformly random molecules (the hit-rate study, Sec. 4);
* ``slab``     -- vapour-liquid slab: FCC liquid layer + random-sequential-
                  addition vapour (uneven cell occupancy, Sec. 5.2);
* ``maxwell``  -- Gaussian velocities at temperature T, zero total momentum,
                  rescaled to T exactly with 3N-3 degrees of freedom.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2510212300


def fcc_sites(ncx: int, ncy: int, ncz: int, a: tuple[float, float, float]) -> np.ndarray:
    """All 4*ncx*ncy*ncz FCC sites of a periodic block of unit cells."""
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    ix, iy, iz = np.meshgrid(np.arange(ncx), np.arange(ncy), np.arange(ncz), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    return sites * np.asarray(a, dtype=np.float64)


def fcc(n: int, rho: float, jitter: float = 0.05, seed: int = SEED_BASE + 1):
    """n molecules on a jittered FCC lattice in a cubic box at density rho.

    The box side is L = (n/rho)^(1/3); the lattice has ceil((n/4)^(1/3)) unit
    cells per side spanning L, and n of its sites are kept by a seeded
    permutation (all of them when n = 4 k^3).  Returns (pos[n,3], box[3]).
    """
    rng = np.random.default_rng(seed)
    L = (n / rho) ** (1.0 / 3.0)
    nc = int(math.ceil((n / 4.0) ** (1.0 / 3.0) - 1e-9))
    sites = fcc_sites(nc, nc, nc, (L / nc,) * 3)
    if len(sites) > n:
        keep = np.sort(rng.permutation(len(sites))[:n])
        sites = sites[keep]
    pos = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    return np.ascontiguousarray(pos), np.array([L, L, L])


def sc(n: int, side: float, seed: int = SEED_BASE + 9):
    """n molecules on a simple cubic lattice in a cubic box of the given side
    (the single-phase start of Sec. 5.1): k = ceil(n^(1/3)) sites per side,
    spacing side/k, n of the k^3 sites kept by a seeded permutation."""
    rng = np.random.default_rng(seed)
    k = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
    g = (np.arange(k) + 0.5) * (side / k)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    sites = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    if len(sites) > n:
        sites = sites[np.sort(rng.permutation(len(sites))[:n])]
    return np.ascontiguousarray(sites), np.array([side, side, side])


def fcc_box(n: int, box, seed: int = SEED_BASE + 11):
    """n molecules on an FCC lattice filling an orthorhombic box: nc_d =
    ceil(L_d / a) unit cells along each side for a = (4 V / n)^(1/3),
    cell edges L_d / nc_d, n of the sites kept by a seeded permutation."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    a = (4.0 * float(np.prod(box)) / n) ** (1.0 / 3.0)
    nc = [int(math.ceil(L / a - 1e-9)) for L in box]
    sites = fcc_sites(nc[0], nc[1], nc[2], tuple(L / k for L, k in zip(box, nc))) + 0.25 * box / np.array(nc)
    if len(sites) > n:
        sites = sites[np.sort(rng.permutation(len(sites))[:n])]
    return np.ascontiguousarray(sites), box.copy()


def lattice(n: int, box, seed: int = SEED_BASE + 10):
    """n molecules on a simple orthorhombic lattice filling an orthorhombic
    box (the homogeneous start of the slab runs of Sec. 5.2): k_d =
    ceil(L_d / a) sites along each side for a = (V / n)^(1/3), spacing
    L_d / k_d, n of the sites kept by a seeded permutation."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    a = (float(np.prod(box)) / n) ** (1.0 / 3.0)
    k = [int(math.ceil(L / a - 1e-9)) for L in box]
    g = [(np.arange(kd) + 0.5) * (L / kd) for kd, L in zip(k, box)]
    x, y, z = np.meshgrid(*g, indexing="ij")
    sites = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    if len(sites) > n:
        sites = sites[np.sort(rng.permutation(len(sites))[:n])]
    return np.ascontiguousarray(sites), box.copy()


def uniform(n: int, box, seed: int = SEED_BASE + 7):
    """n molecules uniformly at random in an orthorhombic box."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    return np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(n, 3)) * box), box.copy()


def rsa(n: int, box, dmin: float = 0.8, lo=None, hi=None, seed: int = SEED_BASE + 8,
        max_tries: int = 200):
    """Random sequential addition: n molecules uniform in the region [lo, hi)
    of a periodic box, each at least dmin (minimum image) from all earlier
    ones.  Returns (pos, box)."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    lo = np.zeros(3) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = box.copy() if hi is None else np.asarray(hi, dtype=np.float64)
    g = np.maximum((box // dmin).astype(int), 1)
    grid = {}
    pts = []
    d2min = dmin * dmin
    for _ in range(n):
        for _t in range(max_tries):
            p = (lo + rng.uniform(0.0, 1.0, 3) * (hi - lo)) % box
            c = tuple((p / box * g).astype(int) % g)
            ok = True
            for off in np.ndindex(3, 3, 3):
                cc = tuple((np.array(c) + np.array(off) - 1) % g)
                for q in grid.get(cc, ()):
                    d = p - q
                    d -= box * np.rint(d / box)
                    if d @ d < d2min:
                        ok = False
                        break
                if not ok:
                    break
            if ok:
                grid.setdefault(c, []).append(p)
                pts.append(p)
                break
        else:
            raise RuntimeError("rsa: region too full for the requested n and dmin")
    return np.ascontiguousarray(np.array(pts)), box.copy()


def slab(lx=30.0, ly=30.0, lz=90.0, z0=30.0, width=30.0, rho_l=0.7, rho_v=0.02,
         jitter=0.05, seed: int = SEED_BASE + 3):
    """Liquid slab z in [z0, z0+width) on a jittered FCC lattice at rho_l,
    vapour elsewhere by random sequential addition at rho_v (molecules closer
    than 1 sigma to any other are rejected).  Returns (pos, box)."""
    rng = np.random.default_rng(seed)
    n_l = int(round(rho_l * lx * ly * width))
    nc = int(math.ceil((n_l / 4.0) ** (1.0 / 3.0) - 1e-9))
    sites = fcc_sites(nc, nc, nc, (lx / nc, ly / nc, width / nc))
    keep = np.sort(rng.permutation(len(sites))[:n_l])
    liquid = sites[keep] + rng.uniform(-jitter, jitter, size=(n_l, 3))
    liquid[:, 2] += z0
    n_v = int(round(rho_v * lx * ly * (lz - width)))
    box = np.array([lx, ly, lz])
    vap = []
    allpts = [liquid]
    tries = 0
    while len(vap) < n_v:
        tries += 1
        if tries > 200 * n_v + 1000:
            raise RuntimeError("slab: vapour insertion failed")
        p = rng.uniform(0.0, 1.0, 3) * np.array([lx, ly, lz - width])
        p[2] = (z0 + width + p[2]) % lz
        cur = np.concatenate(allpts + ([np.array(vap)] if vap else []), axis=0)
        d = cur - p
        d -= box * np.rint(d / box)
        if np.min(np.einsum("ij,ij->i", d, d)) >= 1.0:
            vap.append(p)
    pos = np.concatenate([liquid, np.array(vap)], axis=0)
    return np.ascontiguousarray(pos), box


def maxwell(n: int, T: float, seed: int = SEED_BASE + 2):
    """Gaussian velocities (unit mass), zero momentum, kinetic T exactly."""
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, math.sqrt(T), size=(n, 3))
    v -= v.mean(axis=0, keepdims=True)
    t_now = (v * v).sum() / (3 * n - 3)
    return np.ascontiguousarray(v * math.sqrt(T / t_now))


# Named workloads (positions, box, cutoff parameters).
CONFIGS = {
    # FCC rho 0.6, N = 1000, one evaluation checked against brute force
    "fcc1k": dict(n=1000, rho=0.6, jitter=0.05, seed=SEED_BASE + 1),
    # FCC rho 0.7, N = 32,000 (20^3 unit cells)
    "fcc32k": dict(n=32000, rho=0.7, jitter=0.05, seed=SEED_BASE + 2),
    # FCC rho 0.75, N = 1,000,000 (the throughput workload)
    "fcc1m": dict(n=1000000, rho=0.75, jitter=0.05, seed=SEED_BASE + 4),
}


def make(name: str):
    """Positions and box of a named workload."""
    if name == "slab20k":
        return slab()
    c = CONFIGS[name]
    return fcc(c["n"], c["rho"], c["jitter"], c["seed"])
