"""Localized support-function gradient, Eq. (gradient) of Sec. IV.A, in the
energy mode (FP64).

TEST INFRASTRUCTURE ONLY (oracle).

The target is the band-structure energy Omega = sum_ab K^ab H_ab with the
density kernel K held fixed, so that dOmega/d<phi_b| = sum_d K^bd H|phi_d>.
The Lagrange multipliers of the orthonormality of the Kohn-Sham orbitals
(Sec. IV.A, below Eq. (gradient)) are
    Lambda_ab = <phi_a| sum_c S_bc dOmega/d<phi_c|> = sum_cd H_ad K^dc S_cb,
i.e. Lambda = H K S, and the gradient of support function a is
    g_a = sum_b S_ab dOmega/d<phi_b| - 1/2 sum_b [S^-1 (Lambda + Lambda^T)]_ab |phi_b>
        = sum_d A_ad H|phi_d> - sum_b M_ab |phi_b>,
    A = S K,   M = 1/2 S^-1 (Lambda + Lambda^T),
localized afterwards, g_a <- L^a g_a (Sec. III.A: the gradient of the
localized functional is the projection of the unconstrained one).

Readings (listed in the design notes):
  * S^-1 is taken by its first-order Taylor expansion 2 I - S (the functions
    are nearly orthonormal; the S^-1/2 of App. B is taken the same way);
  * every matrix lives on the overlap pattern P (the pattern of S), H read
    at P's entries, and every product is truncated to P, as in the Fermi
    operator expansion; the Hphi and phi terms of g_a therefore run over the
    functions of row a of P;
  * H|phi_d> is the output of the local-Hamiltonian apply, on d's output
    pattern; L^a keeps the values at a's input pattern (coarse points: the
    scaling coefficient; fine points: the seven wavelets), missing values
    counting as zero.

Parity: pinned in tests/test_oracle_gradient.py by (i) a brute force of the
vector part on one dense global box per function, (ii) the invariant that
for orthonormal functions, a symmetric H and a kernel that commutes with it
the gradient is orthogonal to every function (the Lagrange term removes
exactly the part inside their span), (iii) the Taylor S^-1 against the exact
inverse to second order, and (iv) the truncated products against plain loops
over the pattern.
"""
from __future__ import annotations

import numpy as np

from .locreg import Locreg, points_from_segments


def coefficient_matrices(S, H, K, mask):
    """(A, M) on the pattern: A = (S K)|_P and M = 1/2 ((2 I - S)
    (Lambda + Lambda^T))|_P with Lambda = ((H|_P K)|_P S)|_P.  S is taken by
    its symmetric part; dense (n, n) arrays, mask boolean (n, n)."""
    m = mask.astype(np.float64)
    n = S.shape[0]
    S = 0.5 * (S + S.T) * m
    Hp = H * m
    K = K * m
    A = (S @ K) * m
    lam = ((Hp @ K) * m @ S) * m
    sinv = (2.0 * np.eye(n) - S) * m
    M = 0.5 * (sinv @ (lam + lam.T)) * m
    return A, M


def _index(seg):
    """{(i1, i2, i3): position in the list} of a segment list's points."""
    return {tuple(int(v) for v in p): k for k, p in enumerate(points_from_segments(seg))}


def _values(coef, n_c, cidx, fidx, pts_c, pts_f):
    """A compressed function's values at given coarse points (scaling
    coefficient) and fine points (seven wavelets each); 0 where it has none."""
    coef = np.asarray(coef, np.float64)
    s = np.array([coef[cidx[p]] if p in cidx else 0.0 for p in pts_c])
    d = np.zeros((len(pts_f), 7))
    for r, p in enumerate(pts_f):
        if p in fidx:
            k = fidx[p]
            d[r] = coef[n_c + 7 * k:n_c + 7 * k + 7]
    return s, d


def gradient(lrs, psi, hpsi, A, M, mask, rows=None):
    """g_a = L^a [sum_d A_ad H|phi_d> - sum_b M_ab |phi_b>] for every a (or
    the given rows), in the input layout of a.  psi: per-function
    input-layout vectors; hpsi: per-function output-layout vectors (H|phi>)."""
    n = len(lrs)
    cin = [_index(l.cseg) for l in lrs]
    fin = [_index(l.fseg) for l in lrs]
    cout = [_index(l.ocseg) for l in lrs]
    fout = [_index(l.ofseg) for l in lrs]
    out = []
    for a in (range(n) if rows is None else rows):
        pts_c = [tuple(int(v) for v in p) for p in points_from_segments(lrs[a].cseg)]
        pts_f = [tuple(int(v) for v in p) for p in points_from_segments(lrs[a].fseg)]
        gs = np.zeros(len(pts_c))
        gd = np.zeros((len(pts_f), 7))
        for d in range(n):
            if not mask[a, d]:
                continue
            hs, hd = _values(hpsi[d], lrs[d].on_c, cout[d], fout[d], pts_c, pts_f)
            ps, pd = _values(psi[d], lrs[d].n_c, cin[d], fin[d], pts_c, pts_f)
            gs += A[a, d] * hs - M[a, d] * ps
            gd += A[a, d] * hd - M[a, d] * pd
        out.append(np.concatenate([gs, gd.reshape(-1)]))
    return out
