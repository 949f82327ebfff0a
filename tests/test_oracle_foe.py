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


# ---------------------------------------------------------------------------
# The truncated recursion, pinned by the column form of App. B: column l of
# T^j obeys t_l^0 = e_l, t_l^1 = H~' e_l, t_l^{j+1} = 2 H~' t_l^j - t_l^{j-1};
# localizing the matrices keeps only the entries of column l of the pattern,
# after every step.  Written here one column at a time, with matrix-vector
# products only, so that a mistake in the oracle's matrix form (truncation
# left out of the loop, applied to the wrong index, a wrong sign or factor)
# shows as a difference.
# ---------------------------------------------------------------------------

def _columns(Ht, mask, npl):
    n = Ht.shape[0]
    T = np.zeros((npl + 1, n, n))
    for l in range(n):
        keep = mask[:, l]
        prev = np.zeros(n)
        prev[l] = 1.0
        cur = np.where(keep, Ht[:, l], 0.0)
        T[0][:, l], T[1][:, l] = prev, cur
        for j in range(1, npl):
            nxt = np.where(keep, 2.0 * (Ht @ cur) - prev, 0.0)
            T[j + 1][:, l] = nxt
            prev, cur = cur, nxt
    return T


def _banded(n, w):
    i = np.arange(n)
    return np.abs(i[:, None] - i[None, :]) <= w


def _clusters(m):
    c = np.repeat(np.arange(3), m)
    return np.abs(c[:, None] - c[None, :]) <= 1


@pytest.mark.parametrize("pattern", ["banded", "clusters"])
def test_truncated_recursion_matches_column_form(pattern):
    rng = np.random.default_rng(11)
    mask = _banded(36, 3) if pattern == "banded" else _clusters(12)
    n = mask.shape[0]
    A = _sym(rng, n, 1.0) * mask
    Ht = A / (1.05 * np.max(np.sum(np.abs(A), axis=1)))      # discs inside [-1, 1]
    npl = 60
    want = _columns(Ht, mask, npl)
    got = F.chebyshev_matrices(Ht, npl, mask.astype(float))
    scale = max(1.0, max(np.max(np.abs(t)) for t in want))
    for j in range(npl + 1):
        assert np.max(np.abs(got[j] - want[j])) <= 1e-12 * scale, j
    # the pin is not vacuous: truncating only the final matrices (the planted
    # mistake "no truncation inside the recursion") gives other values
    full = [np.eye(n), Ht.copy()]
    for _ in range(1, npl):
        full.append(2.0 * (Ht @ full[-1]) - full[-2])
    assert np.max(np.abs(full[npl] * mask - want[npl])) > 1e-6


def test_kernel_assembles_from_column_recursion():
    """K of the oracle on a banded pattern equals S^-1/2 K' S^-1/2 (symmetric
    part, truncated) with K' summed column by column from the recursion
    above, at the oracle's mu."""
    rng = np.random.default_rng(12)
    n = 40
    mask = _banded(n, 4)
    m = mask.astype(float)
    S = (np.eye(n) + _sym(rng, n, 0.01)) * mask
    H = (np.diag(np.linspace(-1.0, 2.0, n)) + _sym(rng, n, 0.05)) * mask
    npl, delta = 120, 0.2
    Sh = (1.5 * np.eye(n) - 0.5 * S) * m
    # bounds half a hartree outside the discs: H~' stays inside [-1, 1]
    lo, hi = F.gershgorin(Sh @ H @ Sh)
    K, mu, ebs, (emin, emax) = F.foe(S, H, mask, npl, delta, 15.0, lo - 0.5, hi + 0.5)
    sigma, tau = 2.0 / (emax - emin), 0.5 * (emin + emax)
    Ht = ((Sh @ (sigma * (H - tau * S))) * m @ Sh) * m
    Ht = 0.5 * (Ht + Ht.T)
    assert F.gershgorin(Ht)[0] >= -1.0 and F.gershgorin(Ht)[1] <= 1.0   # no guard here
    T = _columns(Ht, mask, npl)
    c = F.chebyshev_coefficients(lambda x: F.fermi(x / sigma + tau, mu, delta), npl)
    Kp = 0.5 * c[0] * T[0] + np.tensordot(c[1:], T[1:], axes=1)
    want = ((Sh @ Kp) * m @ Sh) * m
    want = 0.5 * (want + want.T)
    assert np.max(np.abs(K - want)) <= 1e-12 * np.max(np.abs(want))
    assert np.all(K[~mask] == 0.0)
    # Tr K' = n_occ at the returned mu
    assert abs(np.trace(Kp) - 15.0) < 1e-9


def _paired_overlap(n, s, rng, noise):
    """S = I plus s on the pairs (2k, 2k + 1), H = -8 I plus a small symmetric
    part, both on the pattern of the pairs: the Gershgorin bounds of
    S^-1/2 H S^-1/2 are tight, and with the Taylor S^-1/2 the scaled H~'
    has an eigenvalue near -1.354, outside [-1, 1]."""
    mask = np.zeros((n, n), bool)
    for k in range(0, n, 2):
        mask[k:k + 2, k:k + 2] = True
    S = np.eye(n)
    for k in range(0, n, 2):
        S[k, k + 1] = S[k + 1, k] = s
    H = (-8.0 * np.eye(n) + _sym(rng, n, noise)) * mask
    return S, H, mask


def test_spectrum_guard_keeps_the_expansion_bounded():
    """Tight Gershgorin bounds with the first-order Taylor S^-1/2 put an
    eigenvalue of H~' outside [-1, 1], where T^i grows like
    cosh(i acosh|x|).  With the guard the recursion runs on the rescaled
    matrix and K equals S^-1/2 f(H~'/sigma + tau) S^-1/2 by eigh (f of the
    unscaled H~', so the rescaling changes nothing but the stability);
    without it K is astronomically wrong."""
    rng = np.random.default_rng(13)
    n = 8
    S, H, mask = _paired_overlap(n, 0.4, rng, 1e-3)
    npl, delta, nocc = 200, 0.5, 4.0
    K, mu, ebs, (emin, emax) = F.foe(S, H, mask, npl, delta, nocc)
    sigma, tau = 2.0 / (emax - emin), 0.5 * (emin + emax)
    Sh = 1.5 * np.eye(n) - 0.5 * S
    Htp = Sh @ (sigma * (H - tau * S)) @ Sh
    assert np.linalg.eigvalsh(Htp)[0] < -1.3          # the case the guard is for
    Kp, lam, f = _eig_kernel(Htp, mu, delta, sigma, tau)
    want = Sh @ Kp @ Sh
    assert np.max(np.abs(K - want)) < 1e-10
    assert abs(np.sum(f) - nocc) < 1e-9
    Kbad = F.foe(S, H, mask, npl, delta, nocc, guard=False)[0]
    assert not np.all(np.abs(Kbad) < 1e3)
