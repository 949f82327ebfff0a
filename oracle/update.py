"""Support-function update step (FP64).

TEST INFRASTRUCTURE ONLY (oracle).

The support functions are optimized by steps along their localized
gradients (paper Sec. III.A: the gradient is projected onto the localization
region, g' = L g; Sec. IV.A: the gradient of a support function is built from
H|phi_a> minus the contribution of the function itself).  The serving
workload uses the simplest such step with a fixed step length eta:
    phi_a <- phi_a - eta (P_La H|phi_a> - H_aa phi_a),
where P_La keeps the coefficients of H|phi_a> (given on the output pattern
L'_a) at the points of the input pattern L_a, and H_aa = <phi_a|H|phi_a>.
"""
from __future__ import annotations

import numpy as np

from .locreg import Locreg, points_from_segments


def restrict_to_input(lr: Locreg, out_coef):
    """P_L: an output-layout vector [s: on_c][d: on_f][7] -> its values at
    the input pattern's points, in the input layout [s: n_c][d: n_f][7]."""
    out_coef = np.asarray(out_coef, np.float64)
    e = lr.ext
    olo = (lr.lo[0] - e, lr.lo[1] - e, lr.lo[2] - e)
    shp = (8, lr.dims[2] + 2 * e, lr.dims[1] + 2 * e, lr.dims[0] + 2 * e)
    box = np.zeros(shp)
    on_c, on_f = lr.on_c, lr.on_f
    poc = points_from_segments(lr.ocseg)
    pof = points_from_segments(lr.ofseg)
    box[0, poc[:, 2] - olo[2], poc[:, 1] - olo[1], poc[:, 0] - olo[0]] = out_coef[:on_c]
    ofine = out_coef[on_c:].reshape(on_f, 7)
    for comp in range(1, 8):
        box[comp, pof[:, 2] - olo[2], pof[:, 1] - olo[1], pof[:, 0] - olo[0]] = ofine[:, comp - 1]
    pic = points_from_segments(lr.cseg)
    pif = points_from_segments(lr.fseg)
    coarse = box[0, pic[:, 2] - olo[2], pic[:, 1] - olo[1], pic[:, 0] - olo[0]]
    fine = np.stack([box[comp, pif[:, 2] - olo[2], pif[:, 1] - olo[1], pif[:, 0] - olo[0]]
                     for comp in range(1, 8)], axis=1).reshape(-1)
    return np.concatenate([coarse, fine])


def update(lr: Locreg, psi, hpsi, h_aa, eta):
    """phi <- phi - eta (P_L H phi - H_aa phi) for one support function."""
    psi = np.asarray(psi, np.float64)
    return psi - eta * (restrict_to_input(lr, hpsi) - h_aa * psi)
