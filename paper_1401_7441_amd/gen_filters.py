"""Generates csrc/wvl_filters.h, the filter tables the HIP kernels use.

Run at build time (``python -m paper_1401_7441_amd.gen_filters``); the
generated header is committed.  Everything is derived here in mpmath from the
mathematics of the least-asymmetric Daubechies family of order 2m = 16 (paper
Sec. II.B: phi and psi vanish outside [1-m, m] = [-7, 8]); no table is typed in.

Derivation (this file's own route):
  * lowpass h: roots of the degree-14 polynomial z^7 P((2 - z - 1/z)/4), with
    P(y) = sum_{k<8} C(7+k, k) y^k; one root of every reciprocal pair {z, 1/z}
    is kept (complex roots with their conjugates), 16 real choices; the one
    whose symbol has the flattest phase (smallest deviation from the chord
    through its end points) is kept, the mirror tie broken towards the larger
    centre of mass sum_k k h_k / sqrt(2) on [-7, 8].
  * g_k = (-1)^k h_{1-k}.
  * moments of phi from the moment generating function
    Phi(t) = prod_{j >= 1} m0(t / 2^j), m0(t) = sum_k h_k e^{k t} / sqrt(2),
    multiplied out as truncated power series.
  * magic filter w_j (j = -7..8) with sum_j w_j j^p = M_p, p = 0..15, through
    the Lagrange basis of the nodes -7..8.
  * kinetic filter a_l (l = -14..14), a_l = int phi(x - l) phi''(x) dx: the
    eigenvector of eigenvalue 1 of l, n -> 4 c_{n-2l} (c = autocorrelation of h),
    by inverse iteration, scaled so that sum_l l^2 a_l = 2.

Fused tables the kernels apply:
  * C_b[n] = sum_k w[n-k] F_b[k], n = -14..16 (F_0 = h, F_1 = g): synthesis
    followed by the magic filter along one axis, f_l = sum_i C_b[l-2i] x_b(i);
    its transpose (analysis after the transposed magic filter) uses the same C.
  * K_ab[j] = sum_{k,k'} F_a[k] a[2j + k' - k] F_b[k'], j = -14..14: the
    second-derivative filter at h/2 seen from the coarse two-level basis
    (output channel a, input channel b), R^T a R along one axis.
"""
from __future__ import annotations

import itertools
import os

import mpmath as mp

DPS = 64
NT = 16
OFF = 7          # h_k, k = -7..8, stored at k + 7


def _poly_mul(p, q):
    out = [0] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _z_polynomial():
    """Ascending coefficients of Q(z) = z^7 P((2 - z - 1/z)/4)."""
    # y = (2 - z - 1/z)/4  =>  z*y = (-z^2 + 2z - 1)/4 ;  z^7 y^k = z^(7-k) (z y)^k
    zy = [mp.mpf(-1) / 4, mp.mpf(2) / 4, mp.mpf(-1) / 4]     # (-1 + 2z - z^2)/4
    Q = [mp.mpf(0)] * 15
    for k in range(8):
        term = [mp.mpf(1)]
        for _ in range(k):
            term = _poly_mul(term, zy)
        term = [mp.mpf(0)] * (7 - k) + term
        c = mp.binomial(7 + k, k)
        for i, v in enumerate(term):
            Q[i] += c * v
    return Q


def _lowpass_candidates():
    Q = _z_polynomial()
    roots = mp.polyroots(Q[::-1], maxsteps=800, extraprec=600)
    inside = [r for r in roots if abs(r) < 1]
    assert len(inside) == 7
    reals = [mp.re(r) for r in inside if abs(mp.im(r)) < mp.mpf(10) ** -40]
    ups = [r for r in inside if mp.im(r) > mp.mpf(10) ** -40]
    cands = []
    groups = [[r] for r in reals] + [[r, mp.conj(r)] for r in ups]
    for flip in itertools.product((False, True), repeat=len(groups)):
        zs = []
        for grp, f in zip(groups, flip):
            zs.extend([1 / z for z in grp] if f else grp)
        poly = [mp.mpf(1)]
        for _ in range(8):
            poly = _poly_mul(poly, [mp.mpf(0.5), mp.mpf(0.5)])
        norm = mp.mpf(1)
        for z in zs:
            poly = _poly_mul(poly, [-z, 1])
            norm *= (1 - z)
        h = [mp.re(c / norm) * mp.sqrt(2) for c in poly]
        cands.append(h)
    return cands


def _chord_phase_deviation(h, npts=400):
    """max over (0, pi) of |phase(H) - chord| after removing the
    ((1+z)/2)^8 factor's exact linear phase."""
    xs = [mp.pi * (i + 0.5) / npts for i in range(npts)]
    ph = []
    last = None
    for x in xs:
        v = sum(hk * mp.expj(-k * x) for k, hk in enumerate(h)) / mp.cos(x / 2) ** 8
        a = mp.arg(v) + 4 * x
        if last is not None:
            a += 2 * mp.pi * mp.nint((last - a) / (2 * mp.pi))
        ph.append(a)
        last = a
    slope = (ph[-1] - ph[0]) / (xs[-1] - xs[0])
    return max(abs(p - ph[0] - slope * (x - xs[0])) for p, x in zip(ph, xs))


def lowpass():
    cands = _lowpass_candidates()
    scored = sorted(((_chord_phase_deviation(h), h) for h in cands), key=lambda t: t[0])
    best = [h for s, h in scored if s - scored[0][0] < mp.mpf(10) ** -20]
    assert len(best) == 2
    com = lambda h: sum((k - OFF) * v for k, v in enumerate(h)) / mp.sqrt(2)
    return max(best, key=com)


def moments(h, pmax=15, depth=240):
    """Taylor coefficients of prod_j m0(t/2^j) -> M_p = p! [t^p]."""
    base = []                          # m0(t) series: sum_p (sum_k h_k k^p/sqrt2) t^p/p!
    for p in range(pmax + 1):
        base.append(sum(v * mp.mpf(k - OFF) ** p for k, v in enumerate(h)) / mp.sqrt(2)
                    / mp.factorial(p))
    prod = [mp.mpf(1)] + [mp.mpf(0)] * pmax
    for j in range(1, depth + 1):
        s = mp.mpf(2) ** (-j)
        fac = [base[p] * s ** p for p in range(pmax + 1)]
        prod = _poly_mul(prod, fac)[:pmax + 1]
    return [prod[p] * mp.factorial(p) for p in range(pmax + 1)]


def magic(mom):
    nodes = list(range(-7, 9))
    w = []
    for j in nodes:
        # Lagrange basis polynomial of node j, ascending coefficients
        poly = [mp.mpf(1)]
        den = mp.mpf(1)
        for k in nodes:
            if k != j:
                poly = _poly_mul(poly, [mp.mpf(-k), mp.mpf(1)])
                den *= (j - k)
        w.append(sum(c * mom[p] for p, c in enumerate(poly)) / den)
    return w


def kinetic(h):
    c = {}
    for j in range(-15, 16):
        c[j] = sum(h[k] * h[k + j] for k in range(NT) if 0 <= k + j < NT)
    n = 29
    A = mp.matrix(n, n)
    for r, l in enumerate(range(-14, 15)):
        for q, m in enumerate(range(-14, 15)):
            A[r, q] = 4 * c.get(m - 2 * l, 0) - (1 if r == q else 0)
    # inverse iteration with a small shift: the eigenvalue-1 eigenvector of 4C
    shift = mp.mpf(10) ** -30
    B = A - shift * mp.eye(n)
    x = mp.matrix([1] * n)
    for _ in range(6):
        x = mp.lu_solve(B, x)
        x = x / mp.norm(x)
    s = sum(mp.mpf(l) ** 2 * x[i] for i, l in enumerate(range(-14, 15)))
    return [2 * x[i] / s for i in range(n)]


def fused(h, g, w, a):
    F = (h, g)
    C = []
    for b in range(2):
        row = []
        for nn in range(-14, 17):
            acc = mp.mpf(0)
            for k in range(-7, 9):
                j = nn - k
                if -7 <= j <= 8:
                    acc += w[j + 7] * F[b][k + 7]
            row.append(acc)
        C.append(row)
    K = [[None, None], [None, None]]
    for ao in range(2):
        for bi in range(2):
            row = []
            for j in range(-14, 15):
                acc = mp.mpf(0)
                for k in range(-7, 9):
                    for kp in range(-7, 9):
                        l = 2 * j + kp - k
                        if -14 <= l <= 14:
                            acc += F[ao][k + 7] * a[l + 14] * F[bi][kp + 7]
                row.append(acc)
            K[ao][bi] = row
    return C, K


def derive():
    with mp.workdps(DPS):
        h = lowpass()
        g = [(-1) ** ((k - OFF) % 2) * h[(1 - (k - OFF)) + OFF] for k in range(NT)]
        mom = moments(h)
        w = magic(mom)
        a = kinetic(h)
        C, K = fused(h, g, w, a)
        return {"h": h, "g": g, "w": w, "a": a, "C": C, "K": K}


def _fmt(vals):
    return ", ".join(float(v).hex() for v in vals)


def f32_nearest(v):
    """The float32 value nearest to the mpmath number v (as a Python float)."""
    import struct
    f = struct.unpack("f", struct.pack("f", float(v)))[0]
    if f == 0.0:
        return 0.0
    x = mp.mpf(f)
    ulp = mp.mpf(2) ** (int(mp.floor(mp.log(abs(x), 2))) - 23)
    best = f
    for cand in (float(x + ulp), float(x - ulp)):
        c32 = struct.unpack("f", struct.pack("f", cand))[0]
        if abs(mp.mpf(c32) - v) < abs(mp.mpf(best) - v):
            best = c32
    return best


def _fmt32(vals):
    return ", ".join(float(f32_nearest(v)).hex() + "f" for v in vals)


def kinetic_row_sums(K):
    """Diagonal completing the scaling-channel difference form of the FP32
    kinetic kernels: they sum sum_{j != 0} K_a0[j] (x_{i+j} - x_i) in double
    with the FP64 taps (the differences of FP32 values are exact there), so
    adding D_a x_i with the row sum D_a = sum_j K_a0[j] gives
    sum_j K_a0[j] x_{i+j}."""
    return [sum(K[a][0]) for a in range(2)]


def write_header(path):
    t = derive()
    lines = [
        "// Generated by paper_1401_7441_amd/gen_filters.py -- do not edit.",
        "// Least-asymmetric Daubechies-16 filters and the fused tables the kernels apply.",
        "#pragma once",
        "",
        "// h_k, g_k, k = -7..8 (index k+7); magic filter w_j, j = -7..8 (index j+7)",
        f"#define WVL_H_F64 {{{_fmt(t['h'])}}}",
        f"#define WVL_G_F64 {{{_fmt(t['g'])}}}",
        f"#define WVL_W_F64 {{{_fmt(t['w'])}}}",
        "// kinetic filter a_l, l = -14..14 (index l+14)",
        f"#define WVL_A_F64 {{{_fmt(t['a'])}}}",
        "// C_b[n], n = -14..16 (index n+14): synthesis then magic filter along one axis",
        f"#define WVL_C0_F64 {{{_fmt(t['C'][0])}}}",
        f"#define WVL_C1_F64 {{{_fmt(t['C'][1])}}}",
        f"#define WVL_C0_F32 {{{_fmt32(t['C'][0])}}}",
        f"#define WVL_C1_F32 {{{_fmt32(t['C'][1])}}}",
        "// K_ab[j], j = -14..14 (index j+14): coarse two-level second-derivative filters",
    ]
    for ao in range(2):
        for bi in range(2):
            lines.append(f"#define WVL_K{ao}{bi}_F64 {{{_fmt(t['K'][ao][bi])}}}")
            lines.append(f"#define WVL_K{ao}{bi}_F32 {{{_fmt32(t['K'][ao][bi])}}}")
    with mp.workdps(DPS):
        D = kinetic_row_sums(t["K"])
    lines += [
        "// FP32 kinetic: row sums D_a = sum_j K_a0[j] (output channel a = 0, 1) that",
        "// complete the scaling-channel difference form to the full filter",
        f"#define WVL_KD_F64 {{{_fmt(D)}}}",
    ]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return t


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    write_header(os.path.join(here, "csrc", "wvl_filters.h"))
