"""Filters of the least-asymmetric Daubechies family of order 2m = 16.

TEST INFRASTRUCTURE ONLY (oracle).  Derived here in mpmath, at 60 significant
digits, from the mathematics; nothing is typed in from a table.

Paper, Sec. II.B: the basis is the orthogonal least-asymmetric Daubechies
family of order 2m = 16; the scaling function phi and the wavelet psi vanish
outside [1-m, m] = [-7, 8].  All filters below are indexed on that window
(the kinetic filter on [-14, 14]).

Conventions (each one is a reading listed in the design notes):
  * phi(x) = sqrt(2) sum_k h_k phi(2x - k),   psi(x) = sqrt(2) sum_k g_k phi(2x - k)
  * g_k = (-1)^k h_{1-k},  k in [-7, 8]
  * M_p = int x^p phi(x) dx  (M_0 = 1)
  * magic filter w_j, j in [-7, 8]:  sum_j w_j j^p = M_p,  p = 0..15
  * kinetic filter a_l = int phi(x - l) phi''(x) dx,  l in [-14, 14]

Selection among the 2^4 spectral factorizations: the one whose phase is
closest to linear (Daubechies' least-asymmetric criterion); the two mirror
images tie, and the tie is broken by the centre of mass M_1 of phi on
[-7, 8], taking the larger one (M_1 ~ 0.84).
"""
from __future__ import annotations

import functools
import itertools

import mpmath as mp

M_HALF = 8                    # m: order 2m = 16
LO, HI = 1 - M_HALF, M_HALF   # support window [-7, 8]
NTAP = HI - LO + 1            # 16
KLO, KHI = -(2 * M_HALF - 2), 2 * M_HALF - 2   # kinetic window [-14, 14]
DPS = 60


def daubechies_y_roots():
    """Roots of P(y) = sum_{k<m} C(m-1+k, k) y^k (Daubechies' polynomial).

    |m0(xi)|^2 = cos^{2m}(xi/2) P(sin^2(xi/2)) is the squared modulus of the
    low-pass symbol of an orthonormal compactly supported scaling function
    with m vanishing wavelet moments.
    """
    with mp.workdps(DPS):
        coeffs = [mp.binomial(M_HALF - 1 + k, k) for k in range(M_HALF)]
        return mp.polyroots(coeffs[::-1], maxsteps=500, extraprec=400)


def _z_pair(y):
    """The two roots z, 1/z of y = (2 - z - 1/z)/4, |z| <= 1 first."""
    b = 1 - 2 * y
    s = mp.sqrt(b * b - 1)
    z1, z2 = b + s, b - s
    if abs(z1) > abs(z2):
        z1, z2 = z2, z1
    return z1, z2


def _h_from_roots(zroots):
    """h_k (k = 0..15) of sqrt(2) ((1+z)/2)^m L(z)/L(1), L(z) = prod (z - z_r)."""
    poly = [mp.mpf(1)]                       # ascending coefficients in z
    def mul(p, q):
        out = [mp.mpc(0)] * (len(p) + len(q) - 1)
        for i, a in enumerate(p):
            for j, b in enumerate(q):
                out[i + j] += a * b
        return out
    for _ in range(M_HALF):
        poly = mul(poly, [mp.mpf(1) / 2, mp.mpf(1) / 2])
    for zr in zroots:
        poly = mul(poly, [-zr, mp.mpf(1)])
    l1 = mp.mpf(1)
    for zr in zroots:
        l1 *= (1 - zr)
    return [mp.re(c / l1) * mp.sqrt(2) for c in poly]


def _phase_nonlinearity(h, npts=513):
    """max |arg H(xi) - slope*xi| over xi in [0, pi] after removing the best
    linear part (least-squares slope through the origin).  H(xi) = sum h_k e^{-ik xi}.
    The linear phase of the ((1+z)/2)^m factor and of any index shift drops out."""
    xs = [mp.pi * i / (npts - 1) for i in range(npts)]
    phases = []
    prev = None
    for x in xs[:-1]:
        val = sum(hk * mp.expj(-k * x) for k, hk in enumerate(h))
        ph = mp.arg(val)
        if prev is not None:
            while ph - prev > mp.pi:
                ph -= 2 * mp.pi
            while ph - prev < -mp.pi:
                ph += 2 * mp.pi
        phases.append(ph)
        prev = ph
    xs = xs[:-1]   # H(pi) = 0: its phase is undefined
    # the factor ((1+z)/2)^m contributes exactly -m*xi/2: remove it, then fit
    res = [p + M_HALF * x / 2 for p, x in zip(phases, xs)]
    num = sum(r * x for r, x in zip(res, xs))
    den = sum(x * x for x in xs)
    slope = num / den
    return max(abs(r - slope * x) for r, x in zip(res, xs))


@functools.lru_cache(maxsize=None)
def factorizations():
    """All 16 real spectral factorizations, as (nonlinearity, M1, h) with
    h indexed k = -7..8 (list position k+7)."""
    with mp.workdps(DPS):
        ys = daubechies_y_roots()
        real = [y for y in ys if abs(mp.im(y)) < mp.mpf(10) ** (-40)]
        cplx = [y for y in ys if mp.im(y) > mp.mpf(10) ** (-40)]
        assert len(real) + 2 * len(cplx) == M_HALF - 1
        out = []
        groups = [("r", mp.re(y)) for y in real] + [("c", y) for y in cplx]
        for choice in itertools.product((0, 1), repeat=len(groups)):
            zs = []
            for (kind, y), pick in zip(groups, choice):
                z = _z_pair(y)[pick]
                if kind == "r":
                    zs.append(mp.re(z))
                else:
                    zs.extend([z, mp.conj(z)])
            h = _h_from_roots(zs)
            nl = _phase_nonlinearity(h)
            m1 = sum((k + LO) * hk for k, hk in enumerate(h)) / mp.sqrt(2)
            out.append((nl, m1, tuple(h)))
        return out


@functools.lru_cache(maxsize=None)
def lowpass_mp():
    """h_k, k = -7..8, of the least-asymmetric factorization (mpmath)."""
    facts = factorizations()
    best = min(f[0] for f in facts)
    ties = [f for f in facts if f[0] - best < mp.mpf(10) ** (-20)]
    assert len(ties) == 2, "least-asymmetric choice must be a mirror pair"
    nl, m1, h = max(ties, key=lambda f: f[1])
    return list(h)


@functools.lru_cache(maxsize=None)
def highpass_mp():
    """g_k = (-1)^k h_{1-k}, k = -7..8."""
    h = lowpass_mp()
    with mp.workdps(DPS):
        return [(-1) ** (k % 2) * h[(1 - k) - LO] for k in range(LO, HI + 1)]


@functools.lru_cache(maxsize=None)
def moments_mp(pmax=15):
    """M_p = int x^p phi(x) dx for p = 0..pmax from the two-scale relation:
    M_p (1 - 2^{-p}) = sqrt(2)/2^{p+1} sum_{q<p} C(p,q) M_q sum_k h_k k^{p-q}."""
    h = lowpass_mp()
    with mp.workdps(DPS):
        mom = [mp.mpf(1)]
        for p in range(1, pmax + 1):
            acc = mp.mpf(0)
            for q in range(p):
                hk = sum(hv * mp.mpf(k + LO) ** (p - q) for k, hv in enumerate(h))
                acc += mp.binomial(p, q) * mom[q] * hk
            mom.append(mp.sqrt(2) / (2 ** (p + 1) - 2) * acc)
        return mom


@functools.lru_cache(maxsize=None)
def wavelet_moments_mp(pmax=15):
    """int x^p psi(x) dx = sqrt(2)/2^{p+1} sum_q C(p,q) M_q sum_k g_k k^{p-q}."""
    g = highpass_mp()
    mom = moments_mp(pmax)
    with mp.workdps(DPS):
        out = []
        for p in range(pmax + 1):
            acc = mp.mpf(0)
            for q in range(p + 1):
                gk = sum(gv * mp.mpf(k + LO) ** (p - q) for k, gv in enumerate(g))
                acc += mp.binomial(p, q) * mom[q] * gk
            out.append(mp.sqrt(2) / 2 ** (p + 1) * acc)
        return out


@functools.lru_cache(maxsize=None)
def magic_mp():
    """Magic filter w_j, j = -7..8: the 16 moment conditions
    sum_j w_j j^p = M_p (p = 0..15), solved as a Vandermonde system."""
    mom = moments_mp(NTAP - 1)
    with mp.workdps(DPS):
        A = mp.matrix(NTAP, NTAP)
        for p in range(NTAP):
            for j in range(NTAP):
                A[p, j] = mp.mpf(j + LO) ** p
        b = mp.matrix([mom[p] for p in range(NTAP)])
        w = mp.lu_solve(A, b)
        return [w[j] for j in range(NTAP)]


@functools.lru_cache(maxsize=None)
def autocorrelation_mp():
    """c_j = sum_k h_k h_{k+j}, j = -15..15 (list position j+15)."""
    h = lowpass_mp()
    out = []
    with mp.workdps(DPS):
        for j in range(-(NTAP - 1), NTAP):
            acc = mp.mpf(0)
            for k in range(NTAP):
                if 0 <= k + j < NTAP:
                    acc += h[k] * h[k + j]
            out.append(acc)
    return out


@functools.lru_cache(maxsize=None)
def kinetic_mp():
    """Second-derivative filter a_l, l = -14..14: the fixed point of
    a_l = 4 sum_j c_j a_{2l+j} (two-scale relation of int phi(x-l) phi''(x) dx)
    normalized by sum_l l^2 a_l = 2 (a quadratic has second derivative 2)."""
    c = autocorrelation_mp()
    n = KHI - KLO + 1
    with mp.workdps(DPS):
        A = mp.matrix(n + 1, n)
        for r, l in enumerate(range(KLO, KHI + 1)):
            for col, nn in enumerate(range(KLO, KHI + 1)):
                j = nn - 2 * l
                cj = c[j + NTAP - 1] if -(NTAP - 1) <= j <= NTAP - 1 else 0
                A[r, col] = 4 * cj - (1 if nn == l else 0)
        for col, nn in enumerate(range(KLO, KHI + 1)):
            A[n, col] = mp.mpf(nn) ** 2
        b = mp.matrix([0] * n + [2])
        sol, res = mp.qr_solve(A, b)
        return [sol[i] for i in range(n)]


def _as_float(v):
    return [float(x) for x in v]


@functools.lru_cache(maxsize=None)
def tables():
    """FP64 tables (nearest doubles of the mpmath values).

    Returns dict with 'h', 'g', 'magic' (index j+7, j = -7..8),
    'kinetic' (index l+14, l = -14..14) and 'moments' (p = 0..15)."""
    return {
        "h": _as_float(lowpass_mp()),
        "g": _as_float(highpass_mp()),
        "magic": _as_float(magic_mp()),
        "kinetic": _as_float(kinetic_mp()),
        "moments": _as_float(moments_mp(15)),
    }
