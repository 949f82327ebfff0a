"""Electronic density on the fine grid (TEST INFRASTRUCTURE ONLY: oracle).

Paper, Sec. II, Eq. (density): with real support functions,
    rho(r) = sum_{a,b} phi_a(r) K^{ab} phi_b(r),
K the density kernel (K^{ab} = sum_i f_i c_i^a c_i^b for orbitals
Psi_i = sum_a c_i^a phi_a, Eq. (expansion)).  The values phi_a(r) are those
on the grid of spacing h/2 that the potential term also uses (Sec. II.B: the
two-level coefficients are synthesized to the h/2 scaling level, the magic
filter gives the point values).  Each function's values live on its fine box:
local fine point l = -14..2N+14 along an axis, stored at index l + 14, sits
at global fine-grid index 2 lo + l + 14 of the (2n + 29)^3 grid.

Parity: fine_values is pinned by the sum rule (its values add up to
2 sqrt(2) times the sum of the coarse scaling coefficients, since the
low-pass filter sums to sqrt(2) per axis and the magic filter to one);
density by the orbital form sum_i f_i Psi_i(r)^2 with each Psi_i synthesized
once on the whole grid.
"""
from __future__ import annotations

import numpy as np

from . import wavelet as W
from .hamiltonian import uncompress
from .locreg import Locreg


def fine_box_shape(lr: Locreg):
    """(z, y, x) shape of the function's fine box."""
    n = lr.dims
    return (2 * n[2] + 29, 2 * n[1] + 29, 2 * n[0] + 29)


def fine_values(lr: Locreg, coef):
    """phi on its fine box [z][y][x]: uncompress, synthesis, magic filter."""
    c8 = uncompress(lr, coef)
    sp = W.synthesis_3d(c8)                 # h/2 scaling coefficients, origin -7
    return W.magic_3d(sp, (-7, -7, -7), (-14, -14, -14), fine_box_shape(lr))


def _rows(kernel, nsf):
    """(a, [(b, K_ab), ...]) per row from a dense array or (rowptr, col, val)."""
    if isinstance(kernel, tuple):
        rowptr, col, val = kernel
        for a in range(nsf):
            yield a, [(int(col[q]), float(val[q])) for q in range(rowptr[a], rowptr[a + 1])]
    else:
        kernel = np.asarray(kernel, np.float64)
        for a in range(nsf):
            yield a, [(b, float(kernel[a, b])) for b in range(nsf) if kernel[a, b] != 0.0]


def density(lrs, coefs, kernel, grid_n, fine=None):
    """rho on the global fine grid (z, y, x), shape 2n + 29 per axis.

    kernel: dense (nsf, nsf) array or CSR (rowptr, col, val); every entry
    K_ab adds K_ab phi_a phi_b on the common part of the two fine boxes."""
    shape = (2 * grid_n[2] + 29, 2 * grid_n[1] + 29, 2 * grid_n[0] + 29)
    if fine is None:
        fine = [fine_values(lr, c) for lr, c in zip(lrs, coefs)]
    rho = np.zeros(shape)
    lo = [tuple(2 * lr.lo[d] for d in (2, 1, 0)) for lr in lrs]       # z, y, x
    for a, row in _rows(kernel, len(lrs)):
        fa = fine[a]
        for b, k in row:
            fb = fine[b]
            g0 = [max(lo[a][d], lo[b][d]) for d in range(3)]
            g1 = [min(lo[a][d] + fa.shape[d], lo[b][d] + fb.shape[d]) for d in range(3)]
            if any(g1[d] <= g0[d] for d in range(3)):
                continue
            sa = tuple(slice(g0[d] - lo[a][d], g1[d] - lo[a][d]) for d in range(3))
            sb = tuple(slice(g0[d] - lo[b][d], g1[d] - lo[b][d]) for d in range(3))
            sg = tuple(slice(g0[d], g1[d]) for d in range(3))
            rho[sg] += k * fa[sa] * fb[sb]
    return rho
