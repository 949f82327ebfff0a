"""Localized local-Hamiltonian application to one support function (FP64).

TEST INFRASTRUCTURE ONLY (oracle).

Paper, Sec. III.B: H|phi_b> = L'^(b) H L^(b) |phi_b>, with H the local part
-1/2 nabla^2 + V of the Kohn-Sham Hamiltonian of Sec. II.A, and L' the
localization projector with the cutoff grown by ext grid points (eight in the
paper).  The operator is the plain definition on the orthonormal two-level
basis of Eq. (Phi):
    T   = exact Galerkin matrix of -1/2 nabla^2, evaluated at the h/2 scaling
          level as -1/2 (2/h)^2 sum_d a *_d  on s' = R c   (R = synthesis);
    V   = R^T W^T diag(V) W R, the magic-filter quadrature (W = magic filter);
    out = P_{L'} R^T (W^T V W + T) R c.
Steps, in the paper's order for the local part:
    uncompress -> synthesis -> magic filter -> potential multiply (e_pot)
    -> transposed magic filter -> + kinetic (e_kin) -> analysis -> compress.
"""
from __future__ import annotations

import numpy as np

from . import wavelet as W
from .locreg import Locreg, points_from_segments


def uncompress(lr: Locreg, coef):
    """Compressed [s: n_c][d: n_f][7] (scaling coefficients of the coarse
    points, then the seven wavelet coefficients of each fine point, points in
    segment order) -> dense (8, N3, N2, N1) box; coefficients absent from the
    pattern are zero."""
    coef = np.asarray(coef, np.float64)
    n_c, n_f = lr.n_c, lr.n_f
    assert coef.size == n_c + 7 * n_f
    box = np.zeros((8, lr.dims[2], lr.dims[1], lr.dims[0]))
    pc = points_from_segments(lr.cseg)
    pf = points_from_segments(lr.fseg)
    lo = lr.lo
    box[0, pc[:, 2] - lo[2], pc[:, 1] - lo[1], pc[:, 0] - lo[0]] = coef[:n_c]
    fine = coef[n_c:].reshape(n_f, 7)
    for comp in range(1, 8):
        box[comp, pf[:, 2] - lo[2], pf[:, 1] - lo[1], pf[:, 0] - lo[0]] = fine[:, comp - 1]
    return box


def compress_out(lr: Locreg, box_out):
    """Dense (8, N3+2e, N2+2e, N1+2e) box on the grown L' box -> compressed
    [s: on_c][d: on_f][7] at the output pattern."""
    e = lr.ext
    olo = (lr.lo[0] - e, lr.lo[1] - e, lr.lo[2] - e)
    pc = points_from_segments(lr.ocseg)
    pf = points_from_segments(lr.ofseg)
    coarse = box_out[0, pc[:, 2] - olo[2], pc[:, 1] - olo[1], pc[:, 0] - olo[0]]
    fine = np.stack([box_out[comp, pf[:, 2] - olo[2], pf[:, 1] - olo[1], pf[:, 0] - olo[0]]
                     for comp in range(1, 8)], axis=1).reshape(-1)
    return np.concatenate([coarse, fine])


def potential_block(lr: Locreg, pot):
    """The support function's block of the global fine-grid potential
    pot[z, y, x]: local fine point l sits at global index 2*lo + l + 14,
    l = -14..2N+14."""
    lo, n = lr.lo, lr.dims
    if pot is None:                      # no external potential
        return np.zeros((2 * n[2] + 29, 2 * n[1] + 29, 2 * n[0] + 29))
    return pot[2 * lo[2]:2 * lo[2] + 2 * n[2] + 29,
               2 * lo[1]:2 * lo[1] + 2 * n[1] + 29,
               2 * lo[0]:2 * lo[0] + 2 * n[0] + 29]


def confinement_block(lr: Locreg, h, a, center):
    """a |r - center|^4 on the function's fine points (paper Sec. IV.A: the
    confining potential of the trace and hybrid modes).  Local fine point l
    sits at (2 lo + l) h/2, l = -14..2N+14."""
    ax = []
    for d in range(3):
        l = np.arange(2 * lr.dims[d] + 29) - 14
        ax.append((2 * lr.lo[d] + l) * (h / 2.0) - center[d])
    r2 = ax[2][:, None, None] ** 2 + ax[1][None, :, None] ** 2 + ax[0][None, None, :] ** 2
    return a * r2 * r2


def apply_local_ham(lr: Locreg, coef, pot, h, kinetic=True, potential=True, conf=0.0,
                    center=None):
    """Returns (hpsi_c, e_kin, e_pot) for one support function.

    coef   : compressed input coefficients on the input pattern (FP64)
    pot    : global fine-grid potential, shape (2n3+29, 2n2+29, 2n1+29), or
             None for no external potential
    h      : coarse grid spacing (bohr)
    conf   : prefactor a of the confining potential a |r - R|^4 added to the
             potential (0: none); R = `center`, else the region's centre.
             e_pot then includes the confinement energy.
    """
    n = lr.dims                      # (N1, N2, N3)
    nz = (n[2], n[1], n[0])          # z, y, x order for array axes
    e = lr.ext
    c8 = uncompress(lr, coef)
    sp = W.synthesis_3d(c8)                          # origin -7
    sp_lo = (-7, -7, -7)
    b_lo = tuple(-2 * e - 7 for _ in range(3))       # analysis needs m = 2i + k
    b_n = tuple(2 * nz[a] + 4 * e + 14 for a in range(3))
    y = np.zeros(b_n)
    e_pot = 0.0
    e_kin = 0.0
    if potential:
        f_lo = (-14, -14, -14)
        f_n = tuple(2 * nz[a] + 29 for a in range(3))
        f = W.magic_3d(sp, sp_lo, f_lo, f_n)
        v = potential_block(lr, pot)
        assert v.shape == f.shape, (v.shape, f.shape)
        if conf:
            v = v + confinement_block(lr, h, conf, lr.center if center is None else center)
        e_pot = float(np.sum(v * f * f))
        y += W.magic_t_3d(v * f, f_lo, b_lo, b_n)
    if kinetic:
        spb = W.embed(sp, sp_lo, b_lo, b_n)
        k = (-0.5 * (2.0 / h) ** 2) * W.laplacian_sum_3d(spb, b_lo)
        e_kin = float(np.sum(spb * k))
        y += k
    out = W.analysis_3d(y, b_lo, (-e, -e, -e), tuple(nz[a] + 2 * e for a in range(3)))
    return compress_out(lr, out), e_kin, e_pot
