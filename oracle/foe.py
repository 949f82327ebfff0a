"""Density kernel by the Fermi operator expansion (TEST INFRASTRUCTURE ONLY:
oracle).

Paper, Sec. IV.B and App. B.  The steps, in the paper's order and notation,
on dense matrices with every product truncated to a pattern P (the
localization of the matrices; here the overlap pattern):
  1. H~ = sigma (H - tau S), sigma = 2 / (eps_max - eps_min),
     tau = (eps_min + eps_max) / 2 (Eq. scale_and_shift_Hamiltonian);
  2. H~' = S^-1/2 H~ S^-1/2 with S^-1/2 from the first-order Taylor
     expansion, (3 I - S) / 2;
  3. K' = c_0/2 I + sum_{i=1..npl} c_i T^i(H~'), the Chebyshev polynomials by
     their recursion T^{j+1} = 2 H~' T^j - T^{j-1}, the c_i the Chebyshev
     coefficients on [-1, 1] of f(eps) = (1 - erf((eps - mu) / delta)) / 2;
  4. mu such that Tr K' is the number of occupied states;
  5. K = S^-1/2 K' S^-1/2 and E_BS = Tr(K H~) / sigma + tau Tr(K S).
Readings (listed in the design notes): S and H enter through their
symmetric parts, H read at P's entries; the symmetric part is taken after
each two-sided product (truncation breaks the symmetry); spectral bounds,
when not given, are the Gershgorin discs of S^-1/2 H S^-1/2.  Spectrum
guard: with the Taylor S^-1/2, S^-1/2 S S^-1/2 is not I, so H~' can reach
outside [-1, 1] even for exact bounds, where T^i grows like
cosh(i acosh|x|).  The Gershgorin discs of H~' are therefore checked; when
they reach outside, the recursion runs on X = (H~' - c I) / r, with [c - r,
c + r] = [min(a, -1), max(b, 1)] for the discs [a, b], and f is taken at
eps(x) = (r x + c) / sigma + tau, so that p(X) still approximates
f(H~' / sigma + tau).  Inside [-1, 1] (c = 0, r = 1) nothing changes.

Parity: pinned by eigendecompositions (tests/test_oracle_foe.py): with S = I
and no truncation, K = f(H) to the expansion error; with a general S and no
truncation, K = S^-1/2 f(H~') S^-1/2 evaluated through eigh, also when the
guard rescales; the truncated recursion against the column form of App. B
(each column t_l^j truncated to column l of the pattern after every step).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erfc


def chebyshev_coefficients(fun, npl, nodes=16384):
    """c_i = (2/pi) int_0^pi fun(cos t) cos(i t) dt, i = 0..npl (midpoint
    rule in t, exact for cosine series of degree below 2 nodes)."""
    t = np.pi * (np.arange(nodes) + 0.5) / nodes
    f = fun(np.cos(t))
    return np.array([2.0 / nodes * np.sum(f * np.cos(i * t)) for i in range(npl + 1)])


def chebyshev_matrices(Ht, npl, mask):
    """T^0 .. T^npl of Ht by the recursion, each truncated to the mask."""
    n = Ht.shape[0]
    T = [np.eye(n), Ht.copy()]
    for _ in range(1, npl):
        T.append((2.0 * (Ht @ T[-1]) - T[-2]) * mask)
    return T


def fermi(eps, mu, delta):
    return 0.5 * erfc((eps - mu) / delta)


def gershgorin(A):
    """Smallest and largest end of the Gershgorin discs of the rows of A."""
    r = np.sum(np.abs(A), axis=1) - np.abs(np.diag(A))
    return float(np.min(np.diag(A) - r)), float(np.max(np.diag(A) + r))


def foe(S, H, mask, npl, delta, n_occ, eps_min=None, eps_max=None, guard=True):
    """Returns (K, mu, E_BS, (eps_min, eps_max)).  S, H dense (n, n); mask
    boolean (n, n), symmetric, holding the diagonal; products truncated to
    it after every multiplication.  guard=False leaves out the spectrum
    guard (for tests that show what it prevents)."""
    m = mask.astype(np.float64)
    S = 0.5 * (S + S.T) * m
    H = 0.5 * (H + H.T) * m
    n = S.shape[0]
    Sh = (1.5 * np.eye(n) - 0.5 * S) * m
    sym = lambda A: 0.5 * (A + A.T)
    if eps_min is None or eps_max is None or eps_min >= eps_max:
        Hp = sym(((Sh @ H) * m @ Sh) * m)
        eps_min, eps_max = gershgorin(Hp)
        if not eps_max > eps_min:
            eps_max = eps_min + 1.0
    sigma = 2.0 / (eps_max - eps_min)
    tau = 0.5 * (eps_min + eps_max)
    Htil = sigma * (H - tau * S)                                   # step 1
    Htp = sym(((Sh @ Htil) * m @ Sh) * m)                          # step 2
    c0, r0 = 0.0, 1.0                                              # spectrum guard
    if guard:
        a, b = gershgorin(Htp)
        if a < -1.0 or b > 1.0:
            glo, ghi = min(a, -1.0), max(b, 1.0)
            c0, r0 = 0.5 * (glo + ghi), 0.5 * (ghi - glo)
            Htp = (Htp - c0 * np.eye(n)) / r0
    T = chebyshev_matrices(Htp, npl, m)                            # step 3
    traces = np.array([np.trace(t) for t in T])

    def coef(mu):
        return chebyshev_coefficients(
            lambda x: fermi((r0 * x + c0) / sigma + tau, mu, delta), npl)

    def trace_kp(mu):
        c = coef(mu)
        return 0.5 * c[0] * traces[0] + float(np.dot(c[1:], traces[1:]))

    lo = (c0 - r0) / sigma + tau - 20.0 * delta                    # step 4
    hi = (c0 + r0) / sigma + tau + 20.0 * delta
    for _ in range(200):
        if hi - lo <= 1e-13 * max(1.0, abs(lo) + abs(hi)):
            break
        mid = 0.5 * (lo + hi)
        if trace_kp(mid) < n_occ:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    c = coef(mu)
    Kp = 0.5 * c[0] * T[0] + sum(c[i] * T[i] for i in range(1, npl + 1))
    K = sym(((Sh @ Kp) * m @ Sh) * m)                              # step 5
    e_bs = float(np.sum(K * Htil)) / sigma + tau * float(np.sum(K * S))
    return K, mu, e_bs, (eps_min, eps_max)
