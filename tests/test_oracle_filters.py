"""Pins of the oracle's filters against facts fixed by the mathematics.

Paper, Sec. II.B: least-asymmetric Daubechies family of order 2m = 16, support
[1-m, m]; its scaling function space reproduces polynomials of low degree.
None of these checks re-derives a filter with the formula that built it."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import filters as F

LO, HI = F.LO, F.HI
mp.mp.dps = F.DPS   # test arithmetic at the derivation's precision


def test_lowpass_orthonormal_and_normalized():
    h = F.lowpass_mp()
    for j in range(-7, 8):
        acc = sum(h[k] * h[k + 2 * j] for k in range(16) if 0 <= k + 2 * j < 16)
        assert abs(acc - (1 if j == 0 else 0)) < mp.mpf(10) ** -45, j
    assert abs(sum(h) - mp.sqrt(2)) < mp.mpf(10) ** -45


def test_highpass_vanishing_moments_and_orthogonal_to_lowpass():
    g = F.highpass_mp()
    h = F.lowpass_mp()
    for p in range(8):                       # m = 8 vanishing moments
        assert abs(sum(gk * mp.mpf(k + LO) ** p for k, gk in enumerate(g))) < mp.mpf(10) ** -40
    # a 9th moment must not vanish (the order is exactly 2m = 16)
    assert abs(sum(gk * mp.mpf(k + LO) ** 8 for k, gk in enumerate(g))) > 1e-3
    for j in range(-7, 8):
        acc = sum(h[k] * g[k + 2 * j] for k in range(16) if 0 <= k + 2 * j < 16)
        assert abs(acc) < mp.mpf(10) ** -45


def test_symbol_squared_modulus_is_daubechies_polynomial():
    """|m0(xi)|^2 = cos^16(xi/2) P(sin^2(xi/2)), P the binomial series."""
    h = F.lowpass_mp()
    for xi in (0.1, 0.7, 1.3, 2.2, 3.0):
        xi = mp.mpf(xi)
        m0 = sum(hk * mp.expj(-k * xi) for k, hk in enumerate(h)) / mp.sqrt(2)
        y = mp.sin(xi / 2) ** 2
        P = sum(mp.binomial(7 + k, k) * y ** k for k in range(8))
        assert abs(abs(m0) ** 2 - mp.cos(xi / 2) ** 16 * P) < mp.mpf(10) ** -40


def test_least_asymmetric_selection():
    """16 factorizations in 8 mirror pairs; the chosen one is the phase-flattest
    pair, well separated from the next, and its mirror has M1' = 1 - M1."""
    facts = sorted(F.factorizations(), key=lambda f: f[0])
    assert len(facts) == 16
    assert facts[1][0] - facts[0][0] < 1e-20
    assert facts[2][0] > facts[0][0] * 1.3
    assert abs(facts[0][1] + facts[1][1] - 1) < 1e-30
    h = F.lowpass_mp()
    m1 = sum((k + LO) * hk for k, hk in enumerate(h)) / mp.sqrt(2)
    assert abs(m1 - max(facts[0][1], facts[1][1])) < 1e-30
    # every factorization is a valid orthonormal filter (same |m0|)
    for _, _, hh in facts:
        assert abs(sum(hh[k] * hh[k + 2] for k in range(14))) < mp.mpf(10) ** -40


def test_moments_satisfy_autocorrelation_identity():
    """Orthonormality of integer translates makes phi's autocorrelation
    interpolating, so Phi(t) Phi(-t) = 1 + O(t^16) for Phi(t) = sum M_q t^q/q!:
    sum_q C(p,q) (-1)^(p-q) M_q M_{p-q} = 0 for 1 <= p <= 15.  (The moments are
    built from the two-scale relation, not from this identity.)"""
    M = F.moments_mp(15)
    for p in range(1, 16):
        acc = sum(mp.binomial(p, q) * (-1) ** (p - q) * M[q] * M[p - q] for q in range(p + 1))
        assert abs(acc) < mp.mpf(10) ** -40, p
    # p = 16 must fail: the degree of exactness is exactly 15
    M16 = F.moments_mp(16)
    acc = sum(mp.binomial(16, q) * (-1) ** (16 - q) * M16[q] * M16[16 - q] for q in range(17))
    assert abs(acc) > 1e-6


def test_magic_filter_reproduces_polynomials_to_degree_15():
    """Exact h/2-level coefficients of a polynomial p (unit spacing) are
    s'_m = sum_q p^(q)(m) M_q / q!;  the magic filter must return p(l) exactly."""
    w = F.magic_mp()
    M = F.moments_mp(15)
    rng = np.random.default_rng(5)
    coef = [mp.mpf(float(c)) for c in rng.standard_normal(16)]
    def p_der(x, q):
        # q-th derivative of sum_k coef[k] (x/5)^k
        acc = mp.mpf(0)
        for k in range(q, 16):
            acc += coef[k] * mp.ff(k, q) * (mp.mpf(x) / 5) ** (k - q) / mp.mpf(5) ** q
        return acc
    for l in (-3, 0, 4, 11):
        sp = {m: sum(p_der(m, q) * M[q] / mp.factorial(q) for q in range(16))
              for m in range(l - HI, l - LO + 1)}
        f = sum(w[j - LO] * sp[l - j] for j in range(LO, HI + 1))
        assert abs(f - p_der(l, 0)) < mp.mpf(10) ** -35 * (1 + abs(p_der(l, 0)))
    assert abs(sum(w) - 1) < mp.mpf(10) ** -45


def test_kinetic_filter_fixed_point_symmetry_and_moments():
    a = F.kinetic_mp()
    c = F.autocorrelation_mp()
    n = len(a)
    for r, l in enumerate(range(F.KLO, F.KHI + 1)):
        rhs = 0
        for col, nn in enumerate(range(F.KLO, F.KHI + 1)):
            j = nn - 2 * l
            if -15 <= j <= 15:
                rhs += 4 * c[j + 15] * a[col]
        assert abs(rhs - a[r]) < mp.mpf(10) ** -40
    for i in range(n):
        assert abs(a[i] - a[n - 1 - i]) < mp.mpf(10) ** -40
    for q in range(0, 16):
        mom = sum(av * mp.mpf(l) ** q for av, l in zip(a, range(F.KLO, F.KHI + 1)))
        target = 2 if q == 2 else 0
        assert abs(mom - target) < mp.mpf(10) ** -35, q


def _phi_hat(xi, h, nprod=48):
    """Fourier transform of phi by the infinite product prod_k m0(xi / 2^k)."""
    k = np.arange(16) + LO
    out = np.ones_like(xi, dtype=complex)
    for j in range(1, nprod + 1):
        x = xi / 2.0 ** j
        out *= (np.exp(-1j * np.outer(x, k)) @ h) / math.sqrt(2)
    return out


def test_kinetic_filter_matches_fourier_integral():
    """a_l = -(1/2pi) int xi^2 |phi_hat(xi)|^2 e^{i l xi} d xi, evaluated by
    quadrature with phi_hat from the infinite product (independent route)."""
    h = np.array(F.tables()["h"])
    a = np.array(F.tables()["kinetic"])
    xi = np.linspace(0.0, 200.0, 400001)
    ph2 = np.abs(_phi_hat(xi, h)) ** 2
    dx = xi[1] - xi[0]
    for l in (0, 1, 2, 5):
        integrand = xi ** 2 * ph2 * np.cos(l * xi)
        val = -(2.0 / (2 * math.pi)) * dx * (integrand.sum() - 0.5 * (integrand[0] + integrand[-1]))
        assert abs(val - a[l + 14]) < 2e-6, (l, val, a[l + 14])


def test_kinetic_symbol_is_minus_xi_squared():
    a = np.array(F.tables()["kinetic"])
    ls = np.arange(F.KLO, F.KHI + 1)
    for xi, tol in ((0.3, 1e-12), (0.5, 2e-9), (1.0, 2e-4)):
        sym = float(np.sum(a * np.cos(ls * xi)))
        assert abs(sym + xi * xi) < tol, (xi, sym + xi * xi)


def test_float_tables_round_the_mp_values():
    t = F.tables()
    for key, src in (("h", F.lowpass_mp()), ("magic", F.magic_mp()),
                     ("kinetic", F.kinetic_mp())):
        for x, y in zip(t[key], src):
            assert x == float(y)
