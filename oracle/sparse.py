"""Sparse overlap and Hamiltonian matrices (TEST INFRASTRUCTURE ONLY: oracle).

Paper, Sec. II.A: S_ab = <phi_a|phi_b> and H_ab = <phi_a|H|phi_b>; Sec. IV.B
stores them compressed, with the pattern given by overlapping localization
regions; App. D computes them as scalar products of compressed support
functions.  On the orthonormal basis of Eq. (Phi) a scalar product is the dot
product of the coefficient vectors, missing coefficients counting as zero.

Pattern (structural): (a, b) is stored for S when the input coarse sets of a
and b share a grid point, and for H when the input coarse set of a shares a
point with the output (L') coarse set of b.  Rows a ascending, columns b
ascending.  The ket of H_ab is (H phi_b) on b's output pattern (Sec. III.B).
"""
from __future__ import annotations

import numpy as np

from .locreg import Locreg, points_from_segments


def _dense(lr_seg_c, lr_seg_f, coef, lo, shape):
    """8-component dense array over the box [lo, lo+shape) (shape = (n3, n2, n1))."""
    out = np.zeros((8,) + tuple(shape))
    pc = points_from_segments(lr_seg_c)
    pf = points_from_segments(lr_seg_f)
    n_c, n_f = len(pc), len(pf)
    coef = np.asarray(coef, np.float64)
    assert coef.size == n_c + 7 * n_f
    if n_c:
        out[0, pc[:, 2] - lo[2], pc[:, 1] - lo[1], pc[:, 0] - lo[0]] = coef[:n_c]
    if n_f:
        fine = coef[n_c:].reshape(n_f, 7)       # [d: n_f][7]
        for comp in range(1, 8):
            out[comp, pf[:, 2] - lo[2], pf[:, 1] - lo[1], pf[:, 0] - lo[0]] = fine[:, comp - 1]
    return out


def _seg_box(segs):
    allseg = np.concatenate([np.asarray(s).reshape(-1, 4) for s in segs])
    lo = (int(allseg[:, 0].min()), int(allseg[:, 2].min()), int(allseg[:, 3].min()))
    hi = (int(allseg[:, 1].max()), int(allseg[:, 2].max()), int(allseg[:, 3].max()))
    return lo, hi


def pair_value(seg_a, coef_a, seg_b, coef_b):
    """Dot product of two compressed functions: seg_x = (coarse, fine) lists."""
    lo, hi = _seg_box([seg_a[0], seg_b[0]])
    shape = (hi[2] - lo[2] + 1, hi[1] - lo[1] + 1, hi[0] - lo[0] + 1)
    da = _dense(seg_a[0], seg_a[1], coef_a, lo, shape)
    db = _dense(seg_b[0], seg_b[1], coef_b, lo, shape)
    return float(np.sum(da * db))


def pair_intersects(cseg_a, cseg_b):
    """True when two coarse segment lists share a grid point."""
    lo, hi = _seg_box([cseg_a, cseg_b])
    shape = (hi[2] - lo[2] + 1, hi[1] - lo[1] + 1, hi[0] - lo[0] + 1)
    ma = np.zeros(shape, bool)
    mb = np.zeros(shape, bool)
    for m, seg in ((ma, cseg_a), (mb, cseg_b)):
        for i1s, i1e, i2, i3 in np.asarray(seg).reshape(-1, 4):
            m[i3 - lo[2], i2 - lo[1], i1s - lo[0]:i1e - lo[0] + 1] = True
    return bool(np.any(ma & mb))


def _bbox(seg):
    seg = np.asarray(seg).reshape(-1, 4)
    return (seg[:, 0].min(), seg[:, 1].max(), seg[:, 2].min(), seg[:, 2].max(),
            seg[:, 3].min(), seg[:, 3].max())


def _boxes_meet(p, q):
    return (p[0] <= q[1] and q[0] <= p[1] and p[2] <= q[3] and q[2] <= p[3]
            and p[4] <= q[5] and q[4] <= p[5])


def pattern(lrs, ket_is_output):
    """CSR (rowptr, col) of the S (ket_is_output = False) or H pattern."""
    bra_box = [_bbox(l.cseg) if l.cseg.size else None for l in lrs]
    ket_box = [_bbox(l.ocseg if ket_is_output else l.cseg)
               if (l.ocseg if ket_is_output else l.cseg).size else None for l in lrs]
    rowptr = [0]
    cols = []
    for a, la in enumerate(lrs):
        for b, lb in enumerate(lrs):
            kseg = lb.ocseg if ket_is_output else lb.cseg
            if bra_box[a] is None or ket_box[b] is None:
                continue
            # disjoint bounding boxes cannot share a point; the decision is
            # the exact set test below
            if not _boxes_meet(bra_box[a], ket_box[b]):
                continue
            if pair_intersects(la.cseg, kseg):
                cols.append(b)
        rowptr.append(len(cols))
    return np.array(rowptr, np.int64), np.array(cols, np.int64)


def matrix(lrs, bra_coefs, ket_coefs, ket_is_output, rows=None):
    """Values of S or H on its pattern.  Returns (rowptr, col, val) for all
    rows, or, if `rows` is given, a dict {(a, b): value} for those rows only."""
    rowptr, col = pattern(lrs, ket_is_output)
    def value(a, b):
        la, lb = lrs[a], lrs[b]
        ket_seg = (lb.ocseg, lb.ofseg) if ket_is_output else (lb.cseg, lb.fseg)
        return pair_value((la.cseg, la.fseg), bra_coefs[a], ket_seg, ket_coefs[b])
    if rows is not None:
        return {(a, int(col[j])): value(a, int(col[j]))
                for a in rows for j in range(rowptr[a], rowptr[a + 1])}
    val = np.array([value(a, int(col[j])) for a in range(len(lrs))
                    for j in range(rowptr[a], rowptr[a + 1])])
    return rowptr, col, val
