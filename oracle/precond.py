"""Preconditioning of support-function gradients (FP64).

TEST INFRASTRUCTURE ONLY (oracle).

Paper Sec. IV.A, Eq. (precond): the localized gradient g of a support
function is preconditioned by approximately solving
    (-1/2 nabla^2 + a (r - R)^4 - eps) x = -g
on the function's localization region, with eps an approximate Lagrange
multiplier.  Readings: the operator is restricted to the input pattern on
both sides, A = P_L (T + C) P_L - eps (symmetric); eps above 0 is taken as 0
so that A stays positive definite; the approximate solve is a fixed number
of conjugate-gradient steps from x = 0 (the paper asks only for an
approximate solution and names no method).
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import apply_local_ham
from .locreg import Locreg
from .update import restrict_to_input


def apply_operator(lr: Locreg, x, h, conf, eps):
    """A x = P_L (T + a |r - R|^4) P_L x - min(eps, 0) x."""
    hx, _, _ = apply_local_ham(lr, x, None, h, kinetic=True, potential=bool(conf), conf=conf)
    return restrict_to_input(lr, hx) - min(eps, 0.0) * np.asarray(x, np.float64)


def precondition(lr: Locreg, g, h, conf, eps, niter):
    """`niter` conjugate-gradient steps on A x = -g from x = 0."""
    g = np.asarray(g, np.float64)
    x = np.zeros_like(g)
    r = -g.copy()
    p = r.copy()
    rr = float(r @ r)
    for _ in range(niter):
        ap = apply_operator(lr, p, h, conf, eps)
        pap = float(p @ ap)
        al = rr / pap if (pap > 0.0 and rr > 0.0) else 0.0
        x = x + al * p
        r = r - al * ap
        rr_new = float(r @ r)
        be = rr_new / rr if rr > 0.0 else 0.0
        p = r + be * p
        rr = rr_new
    return x
