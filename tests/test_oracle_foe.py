"""Pins of the Fermi-operator-expansion oracle (paper Sec. IV.B, App. B)
against eigendecompositions, which reach the same matrices by another route:

* S = I, no truncation: K = f(H) = V f(lambda) V^T, Tr K = n_occ and
  E_BS = sum_i f(lambda_i) lambda_i (the Chebyshev recursion, the
  coefficients, the scaling and shift and the mu search);
* general S, no truncation: K = S^-1/2 f(H~') S^-1/2 with the first-order
  Taylor S^-1/2, f evaluated through eigh of H~' (the transforms around the
  expansion);
* a banded pattern: K vanishes off the pattern and is symmetric, and its
  trace condition holds.
"""
import numpy as np
import pytest

from oracle import foe as F


def _sym(rng, n, scale):
    a = rng.standard_normal((n, n)) * scale
    return 0.5 * (a + a.T)


def _eig_kernel(A, mu, delta, sigma=1.0, tau=0.0):
    lam, V = np.linalg.eigh(A)
    f = F.fermi(lam / sigma + tau, mu, delta)
    return (V * f) @ V.T, lam, f


@pytest.mark.parametrize("given_bounds", [True, False])
def test_identity_overlap_gives_fermi_function_of_h(given_bounds):
    rng = np.random.default_rng(5)
    n = 30
    H = np.diag(np.linspace(-0.9, 0.9, n)) + _sym(rng, n, 0.02)
    S = np.eye(n)
    mask = np.ones((n, n), bool)
    lam = np.linalg.eigvalsh(H)
    b = (lam[0] - 0.05, lam[-1] + 0.05) if given_bounds else (None, None)
    K, mu, ebs, _ = F.foe(S, H, mask, npl=240, delta=0.08, n_occ=11.0,
                          eps_min=b[0], eps_max=b[1])
    want, lam, f = _eig_kernel(H, mu, 0.08)
    assert np.max(np.abs(K - want)) < 1e-11
    assert abs(np.sum(f) - 11.0) < 1e-9
    assert abs(ebs - np.sum(f * lam)) < 1e-10


def test_general_overlap_matches_eigen_route():
    rng = np.random.default_rng(6)
    n = 24
    S = np.eye(n) + _sym(rng, n, 0.01)
    H = np.diag(np.linspace(-2.0, 3.0, n)) + _sym(rng, n, 0.05)
    mask = np.ones((n, n), bool)
    K, mu, ebs, (emin, emax) = F.foe(S, H, mask, npl=300, delta=0.15, n_occ=9.5)
    sigma, tau = 2.0 / (emax - emin), 0.5 * (emin + emax)
    Sh = 1.5 * np.eye(n) - 0.5 * S
    Htil = sigma * (H - tau * S)
    Kp, lam, f = _eig_kernel(Sh @ Htil @ Sh, mu, 0.15, sigma, tau)
    want = Sh @ Kp @ Sh
    assert np.max(np.abs(K - want)) < 1e-10 * np.max(np.abs(want))
    assert abs(np.sum(f) - 9.5) < 1e-9
    assert abs(ebs - (np.sum(want * Htil) / sigma + tau * np.sum(want * S))) < 1e-9
    # the bounds enclose the spectrum of S^-1/2 H S^-1/2
    ev = np.linalg.eigvalsh(Sh @ H @ Sh)
    assert emin <= ev[0] + 1e-12 and ev[-1] <= emax + 1e-12


def test_banded_pattern_truncates_and_keeps_the_trace():
    rng = np.random.default_rng(7)
    n = 40
    idx = np.arange(n)
    mask = np.abs(idx[:, None] - idx[None, :]) <= 4
    S = (np.eye(n) + _sym(rng, n, 0.01)) * mask
    H = (np.diag(np.linspace(-1.0, 2.0, n)) + _sym(rng, n, 0.05)) * mask
    K, mu, ebs, (emin, emax) = F.foe(S, H, mask, npl=120, delta=0.2, n_occ=15.0)
    assert np.all(K[~mask] == 0.0)
    assert np.array_equal(K, K.T)
    sigma, tau = 2.0 / (emax - emin), 0.5 * (emin + emax)
    Sh = (1.5 * np.eye(n) - 0.5 * S) * mask
    Ht = 0.5 * (((Sh @ (sigma * (H - tau * S))) * mask @ Sh) * mask)
    Ht = Ht + Ht.T
    T = F.chebyshev_matrices(Ht, 120, mask.astype(float))
    c = F.chebyshev_coefficients(lambda x: F.fermi(x / sigma + tau, mu, 0.2), 120)
    tr = 0.5 * c[0] * n + sum(c[i] * np.trace(T[i]) for i in range(1, 121))
    assert abs(tr - 15.0) < 1e-9
