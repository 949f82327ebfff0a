"""Seeded synthetic inputs for the local-Hamiltonian path.

This module holds random draws and data layout only: it contains none of the
method's arithmetic (no filters, no localization rule, no operator).  Both the
oracle and the GPU library consume what it produces, so that both see the same
numbers.  Segment lists come from a builder (the oracle's or the library's);
this module only draws values on the points those lists name.

Workloads (the paper measures on molecules whose geometries and pseudopotentials
are not available; these synthetic stand-ins have the shapes of its
localization regions: radii of 5-7 bohr at h = 0.45 bohr, fine regions of a
few bohr around each centre, a smooth local potential of Gaussian wells):

  single   one support function, FP64, 20^3 coarse box at h = 0.5 bohr, the
           fine region the inner 10^3; N(0,1) coefficients times a Gaussian
           envelope (sigma 3 bohr) at the box centre; potential = 8 Gaussian
           wells (depth U(-2,0) Ha, width U(0.5,1.5) bohr) on the 69^3 fine grid.
  batch1k  1,000 support functions, centres uniform in a 30 bohr cube,
           R ~ U(5,7) bohr, h = 0.45, fine radius 3.5 bohr, L' margin 8;
           coefficients N(0,1) x exp(-r^2 / (2 (R/2)^2)), normalized per
           function; potential = one Gaussian well per support function.
  gpu16k   16,000 support functions, centres uniform in a 110 bohr cube
           (a binomial stand-in for a Poisson process), otherwise as batch1k.
  sweep2k  2,000 support functions whose cubic box edge E ~ U{16..48}
           coarse points, R = (E-1) h / 2, fine radius min(3.5, R),
           density 0.012 centres per bohr^3.
  serve    independent systems of 50-4,000 support functions (log-uniform),
           R ~ U(4.5, 7.5) bohr, density 0.012 per bohr^3.

Seeds: numpy PCG64 streams spawned from SeedSequence([14017441 + k, ...]),
one stream for geometry, one per support function for coefficients, one for
the potential, so that any subset of support functions can be regenerated
alone.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BASE_SEED = 14017441

WORKLOADS = {"single": 1, "batch1k": 2, "gpu16k": 3, "serve": 4, "sweep2k": 5}


def _rng(k, *path):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED + k, *path])))


@dataclass
class Geometry:
    """Global grid and per-support-function localization parameters."""
    h: float
    grid_n: tuple          # global coarse points (n1, n2, n3)
    centers: np.ndarray    # (nsf, 3) bohr, in grid coordinates (origin at index 0)
    radii: np.ndarray      # (nsf,)
    fine_radii: np.ndarray  # (nsf,)
    ext: int
    domain_lo: np.ndarray  # bohr, the cube the centres were drawn in
    domain_hi: np.ndarray
    workload: int
    envelope_sigma: np.ndarray  # (nsf,) Gaussian envelope width of the coefficients


def _placed(k, centers_raw, radii, h, ext, side):
    margin = float(np.max(radii)) + (ext + 2) * h
    centers = centers_raw + margin
    n = int(math.ceil((side + 2 * margin) / h)) + 1
    return centers, (n, n, n), np.full(3, margin), np.full(3, margin + side)


def geometry(workload, nsf=None, seed_offset=0):
    """Geometry of a named workload (see module docstring).  `nsf` overrides
    the support-function count (for reduced test cases)."""
    k = WORKLOADS[workload] if isinstance(workload, str) else int(workload)
    rng = _rng(k, 0, seed_offset)
    if k == 1:
        h = 0.5
        c = np.array([[h * 19 / 2] * 3])
        return Geometry(h=h, grid_n=(20, 20, 20), centers=c, radii=np.array([0.0]),
                        fine_radii=np.array([0.0]), ext=0, domain_lo=np.zeros(3),
                        domain_hi=np.full(3, h * 19), workload=k,
                        envelope_sigma=np.array([3.0]))
    h = 0.45
    ext = 8
    if k in (2, 3):
        nsf = nsf or (1000 if k == 2 else 16000)
        side = 30.0 if k == 2 else 110.0
        if nsf is not None and k == 2 and nsf != 1000:
            side = 30.0 * (nsf / 1000.0) ** (1.0 / 3.0)
        if nsf is not None and k == 3 and nsf != 16000:
            side = 110.0 * (nsf / 16000.0) ** (1.0 / 3.0)
        raw = rng.uniform(0.0, side, size=(nsf, 3))
        radii = rng.uniform(5.0, 7.0, size=nsf)
        fine = np.full(nsf, 3.5)
    elif k == 4:
        nsf = nsf or int(math.floor(math.exp(rng.uniform(math.log(50), math.log(4000)))))
        side = (nsf / 0.012) ** (1.0 / 3.0)
        raw = rng.uniform(0.0, side, size=(nsf, 3))
        radii = rng.uniform(4.5, 7.5, size=nsf)
        fine = np.full(nsf, 3.5)
    elif k == 5:
        nsf = nsf or 2000
        side = (nsf / 0.012) ** (1.0 / 3.0)
        raw = rng.uniform(0.0, side, size=(nsf, 3))
        edge = rng.integers(16, 49, size=nsf)
        radii = (edge - 1) * h / 2.0
        fine = np.minimum(3.5, radii)
    else:
        raise ValueError(workload)
    centers, n, dlo, dhi = _placed(k, raw, radii, h, ext, side)
    return Geometry(h=h, grid_n=n, centers=centers, radii=radii, fine_radii=fine, ext=ext,
                    domain_lo=dlo, domain_hi=dhi, workload=k, envelope_sigma=radii / 2.0)


def coefficients(geom: Geometry, sf, points_c, points_f, smooth=False, normalize=True):
    """Compressed coefficients [s: n_c][d: n_f][7] of support function `sf`
    (the seven wavelet coefficients of a fine point are contiguous).

    points_c / points_f: (n, 3) global coarse points (i1, i2, i3) of the input
    coarse / fine pattern, in segment order.  Each value is N(0,1) times the
    Gaussian envelope exp(-|h i - c|^2 / (2 sigma^2)) (`smooth`: the envelope
    alone, scaling coefficients only).  Normalized to unit norm unless told not."""
    rng = _rng(geom.workload, 1, int(sf))
    c = geom.centers[sf]
    sig = float(geom.envelope_sigma[sf])
    def env(p):
        r = geom.h * np.asarray(p, np.float64) - c
        return np.exp(-np.sum(r * r, axis=1) / (2.0 * sig * sig))
    ec = env(points_c)
    ef = env(points_f)
    nc, nf = len(points_c), len(points_f)
    if smooth:
        out = np.concatenate([ec, np.zeros(7 * nf)])
    else:
        # draws per (component, point) as before; stored point-major
        out = np.concatenate([rng.standard_normal(nc) * ec,
                              (rng.standard_normal((7, nf)) * ef[None, :]).T.ravel()])
    if normalize:
        nrm = math.sqrt(float(np.dot(out, out)))
        if nrm > 0:
            out = out / nrm
    return out


def flat_coefficients(geom: Geometry, n, seed=0):
    """n coefficients N(0, 1/n) from one stream per system (stream 3, then
    `seed`): a fast stand-in where only the sizes matter (the serving
    measurement)."""
    rng = _rng(geom.workload, 3, seed)
    return rng.standard_normal(n) / math.sqrt(max(1, n))


def potential_params(geom: Geometry, ngauss=None):
    """Gaussian wells: centres uniform in the domain, depth U(-2, 0) Ha,
    width U(0.5, 1.5) bohr.  One well per support function unless given."""
    rng = _rng(geom.workload, 2)
    ng = ngauss or (8 if geom.workload == 1 else len(geom.centers))
    cen = rng.uniform(geom.domain_lo, geom.domain_hi, size=(ng, 3))
    amp = rng.uniform(-2.0, 0.0, size=ng)
    wid = rng.uniform(0.5, 1.5, size=ng)
    return cen, amp, wid


def fine_grid_shape(grid_n):
    """Global fine grid (z, y, x) shape: 2n + 29 points per axis."""
    return (2 * grid_n[2] + 29, 2 * grid_n[1] + 29, 2 * grid_n[0] + 29)


def potential(geom: Geometry, device="cpu", dtype=None, params=None, cutoff=6.0):
    """Global fine-grid potential V[z, y, x] (torch tensor, float64 by default).

    Global fine index p sits at (p - 14) * h / 2 bohr.  Each well is summed
    over the points within `cutoff` widths of its centre (beyond that it is
    below 2e-8 of its depth)."""
    import torch
    dtype = dtype or torch.float64
    cen, amp, wid = params if params is not None else potential_params(geom)
    shp = fine_grid_shape(geom.grid_n)
    v = torch.zeros(shp, dtype=torch.float64, device=device)
    hf = geom.h / 2.0
    for g in range(len(amp)):
        r = cutoff * wid[g]
        idx = []
        for ax in range(3):                # x, y, z
            n_ax = shp[2 - ax]
            p0 = max(0, int(math.floor((cen[g, ax] - r) / hf)) + 14)
            p1 = min(n_ax - 1, int(math.ceil((cen[g, ax] + r) / hf)) + 14)
            idx.append((p0, p1))
        if any(p1 < p0 for p0, p1 in idx):
            continue
        e = []
        for ax in range(3):
            p = torch.arange(idx[ax][0], idx[ax][1] + 1, dtype=torch.float64, device=device)
            x = (p - 14) * hf - float(cen[g, ax])
            e.append(torch.exp(-(x * x) / (2.0 * float(wid[g]) ** 2)))
        blk = float(amp[g]) * e[2][:, None, None] * e[1][None, :, None] * e[0][None, None, :]
        v[idx[2][0]:idx[2][1] + 1, idx[1][0]:idx[1][1] + 1, idx[0][0]:idx[0][1] + 1] += blk
    return v.to(dtype)


def single_box():
    """The single-function workload's box: lo (0,0,0), 20^3 coarse points,
    fine region the inner 10^3 (coarse indices 5..14)."""
    return (0, 0, 0), (20, 20, 20), (5, 5, 5), (14, 14, 14)


def write_geometry(workload, path, nsf=None):
    """Write a workload's geometry as a flat little-endian file for native
    drivers: int32 nsf, int32 grid_n[3], int32 ext, int32 0, float64 h, then
    float64 centers[nsf][3], radii[nsf], fine_radii[nsf]."""
    g = geometry(workload, nsf=nsf)
    m = len(g.radii)
    with open(path, "wb") as f:
        f.write(np.array([m, *g.grid_n, g.ext, 0], dtype="<i4").tobytes())
        f.write(np.array([g.h], dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(g.centers, dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(g.radii, dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(g.fine_radii, dtype="<f8").tobytes())

