"""Localization regions and segment lists (TEST INFRASTRUCTURE ONLY: oracle).

Paper, Sec. III: the projector L^(alpha) keeps the coefficients of grid points
within R_cut of the centre R_alpha (a Heaviside function of the distance);
Sec. III.B: H|phi_b> = L'^(b) H L^(b) |phi_b>, where L' uses R_cut plus eight
grid points.  Sec. II.B: the simulation box has its origin in a corner, so
global coarse indices are >= 0 and point i sits at h*i.

Readings (listed in the design notes):
  * membership is inclusive: (h*i1-X)^2 + (h*i2-Y)^2 + (h*i3-Z)^2 <= R*R,
    evaluated in FP64 in that order (numpy performs no FMA contraction);
  * the input box L is the bounding box of the coarse sphere points;
  * the output pattern L' = points with distance^2 <= (R + ext*h)^2 that lie
    in the input box grown by ext points on every side and in the grid;
  * the input fine set = coarse set points within the fine radius; the output
    fine set = L' points that belong to the union F of all input fine sets;
  * a segment = a maximal run of consecutive i1 at fixed (i2, i3), inclusive
    ends; segments are sorted by (i3, i2, i1_start).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Locreg:
    lo: tuple            # (x, y, z) global coarse index of the input box origin
    dims: tuple          # (N1, N2, N3)
    ext: int
    cseg: np.ndarray     # (k, 4) int64 rows (i1s, i1e, i2, i3), input coarse
    fseg: np.ndarray     # input fine
    ocseg: np.ndarray    # output (L') coarse
    ofseg: np.ndarray    # output fine
    center: tuple = (0.0, 0.0, 0.0)
    radius: float = 0.0

    @property
    def n_c(self):
        return int(seg_count(self.cseg))

    @property
    def n_f(self):
        return int(seg_count(self.fseg))

    @property
    def on_c(self):
        return int(seg_count(self.ocseg))

    @property
    def on_f(self):
        return int(seg_count(self.ofseg))


def seg_count(seg):
    seg = np.asarray(seg)
    if seg.size == 0:
        return 0
    return int(np.sum(seg[:, 1] - seg[:, 0] + 1))


def segments_from_mask(mask, origin):
    """mask[z, y, x] on the box whose global origin is origin = (x, y, z)
    -> (k, 4) array of maximal i1 runs (i1s, i1e, i2, i3), sorted by
    (i3, i2, i1s)."""
    mask = np.asarray(mask, bool)
    out = []
    n3, n2, n1 = mask.shape
    for z in range(n3):
        for y in range(n2):
            row = mask[z, y]
            x = 0
            while x < n1:
                if row[x]:
                    x0 = x
                    while x < n1 and row[x]:
                        x += 1
                    out.append((origin[0] + x0, origin[0] + x - 1,
                                origin[1] + y, origin[2] + z))
                else:
                    x += 1
    return np.array(out, dtype=np.int64).reshape(-1, 4)


def mask_from_segments(seg, origin, shape):
    """Inverse of segments_from_mask on a box (shape given as (n3, n2, n1))."""
    m = np.zeros(shape, bool)
    for i1s, i1e, i2, i3 in np.asarray(seg).reshape(-1, 4):
        m[i3 - origin[2], i2 - origin[1], i1s - origin[0]:i1e - origin[0] + 1] = True
    return m


def points_from_segments(seg):
    """Global coarse points of a segment list, in compressed (segment) order,
    as an (n, 3) array of (i1, i2, i3)."""
    pts = []
    for i1s, i1e, i2, i3 in np.asarray(seg).reshape(-1, 4):
        for i1 in range(i1s, i1e + 1):
            pts.append((i1, i2, i3))
    return np.array(pts, dtype=np.int64).reshape(-1, 3)


def _dist2(h, c, i1, i2, i3):
    dx = h * i1.astype(np.float64) - c[0]
    dy = h * i2.astype(np.float64) - c[1]
    dz = h * i3.astype(np.float64) - c[2]
    return (dx * dx + dy * dy) + dz * dz


def _ball(h, c, r, grid_n, box_lo, box_hi):
    """Mask of grid points within distance r of c, over the candidate box
    [box_lo, box_hi] (clipped to the grid); returns (mask[z,y,x], lo)."""
    lo = [max(0, box_lo[a]) for a in range(3)]
    hi = [min(grid_n[a] - 1, box_hi[a]) for a in range(3)]
    if any(hi[a] < lo[a] for a in range(3)):
        return np.zeros((0, 0, 0), bool), lo
    i3, i2, i1 = np.meshgrid(np.arange(lo[2], hi[2] + 1), np.arange(lo[1], hi[1] + 1),
                             np.arange(lo[0], hi[0] + 1), indexing="ij")
    r2 = r * r
    return _dist2(h, c, i1, i2, i3) <= r2, lo


class SphereSet:
    """Coarse and fine sets of spheres (coarse radius R, fine radius r_f) and
    the union F of the fine sets; locreg(k) builds function k's Locreg with
    L' radius R + ext*h (see the module docstring for the exact rules)."""

    def __init__(self, h, grid_n, centers, radii, fine_radii, ext):
        self.h, self.grid_n, self.ext = h, grid_n, ext
        self.centers, self.radii = centers, radii
        nsf = len(centers)
        self.coarse = []
        for k in range(nsf):
            c = [float(v) for v in centers[k]]
            R = float(radii[k])
            cand_lo = [int(np.floor((c[a] - R) / h)) - 1 for a in range(3)]
            cand_hi = [int(np.ceil((c[a] + R) / h)) + 1 for a in range(3)]
            m, mlo = _ball(h, c, R, grid_n, cand_lo, cand_hi)
            if not m.any():
                raise ValueError(f"support function {k}: empty localization region")
            zz, yy, xx = np.nonzero(m)
            lo = (mlo[0] + int(xx.min()), mlo[1] + int(yy.min()), mlo[2] + int(zz.min()))
            hi = (mlo[0] + int(xx.max()), mlo[1] + int(yy.max()), mlo[2] + int(zz.max()))
            m = m[lo[2] - mlo[2]:hi[2] - mlo[2] + 1, lo[1] - mlo[1]:hi[1] - mlo[1] + 1,
                  lo[0] - mlo[0]:hi[0] - mlo[0] + 1]
            self.coarse.append((lo, hi, m))
        # input fine sets and their union F
        self.F = np.zeros((grid_n[2], grid_n[1], grid_n[0]), bool)
        self.fine = []
        for k, (lo, hi, m) in enumerate(self.coarse):
            c = [float(v) for v in centers[k]]
            fm, flo = _ball(h, c, float(fine_radii[k]), grid_n, lo, hi)
            fm = fm & m
            self.fine.append(fm)
            self.F[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] |= fm

    def coarse_set(self, k, output=False):
        """(mask[z, y, x], origin (x, y, z)) of function k's input coarse set,
        or of its output (L') coarse set."""
        if not output:
            lo, hi, m = self.coarse[k]
            return m, tuple(lo)
        lo, hi, m = self.coarse[k]
        c = [float(v) for v in self.centers[k]]
        Rp = float(self.radii[k]) + self.ext * self.h
        om, omlo = _ball(self.h, c, Rp, self.grid_n, [lo[a] - self.ext for a in range(3)],
                         [hi[a] + self.ext for a in range(3)])
        return om, tuple(omlo)

    def locreg(self, k):
        h, grid_n, ext, F = self.h, self.grid_n, self.ext, self.F
        lo, hi, m = self.coarse[k]
        c = [float(v) for v in self.centers[k]]
        om, omlo = self.coarse_set(k, output=True)
        if om.size:
            ofm = om & F[omlo[2]:omlo[2] + om.shape[0], omlo[1]:omlo[1] + om.shape[1],
                         omlo[0]:omlo[0] + om.shape[2]]
        else:
            ofm = om
        return Locreg(
            lo=tuple(lo), dims=tuple(hi[a] - lo[a] + 1 for a in range(3)), ext=int(ext),
            cseg=segments_from_mask(m, lo), fseg=segments_from_mask(self.fine[k], lo),
            ocseg=segments_from_mask(om, omlo), ofseg=segments_from_mask(ofm, omlo),
            center=tuple(c), radius=float(self.radii[k]))


def sphere_locregs(h, grid_n, centers, radii, fine_radii, ext):
    """Locregs of spheres: coarse set radius R, fine set radius r_f, L' radius
    R + ext*h (see module docstring for the exact rules)."""
    s = SphereSet(h, grid_n, centers, radii, fine_radii, ext)
    return [s.locreg(k) for k in range(len(centers))]


def box_locreg(lo, dims, fine_lo, fine_hi, ext=0):
    """A rectangular locreg: coarse set = the whole box, fine set = the
    sub-box [fine_lo, fine_hi] (inclusive, global), output = input (ext = 0)."""
    assert ext == 0
    m = np.ones((dims[2], dims[1], dims[0]), bool)
    fm = np.zeros_like(m)
    fm[fine_lo[2] - lo[2]:fine_hi[2] - lo[2] + 1, fine_lo[1] - lo[1]:fine_hi[1] - lo[1] + 1,
       fine_lo[0] - lo[0]:fine_hi[0] - lo[0] + 1] = True
    cs = segments_from_mask(m, lo)
    fs = segments_from_mask(fm, lo)
    return Locreg(lo=tuple(lo), dims=tuple(dims), ext=0, cseg=cs, fseg=fs,
                  ocseg=cs.copy(), ofseg=fs.copy())
