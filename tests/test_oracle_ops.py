"""Pins of the oracle's operators (not its filters) against closed forms,
invariants and brute force.

Paper, Sec. II.B (orthonormal two-level basis, Eq. (Phi)), Sec. III
(localization projector), Sec. III.B (H|phi> = L' H L |phi>), Sec. II.A
(S_ab, H_ab)."""
import math

import mpmath as mp
import numpy as np
import pytest

import inputs
from oracle import filters as F
from oracle import hamiltonian as Hm
from oracle import locreg as LR
from oracle import sparse as SP
from oracle import wavelet as W


# ----------------------------------------------------------------------------
# exact projections of a Gaussian (test helper, independent of the operators)
# ----------------------------------------------------------------------------

def gauss_projection_1d(h, sigma, x0, n, qmax=60):
    """(s_i, d_i), i = 0..n-1, of g(x) = exp(-(x-x0)^2/(2 sigma^2)) on the
    level-h basis phi^h_i(x) = h^{-1/2} phi(x/h - i) (and psi likewise):
    s_i = h^{1/2} sum_q h^q g^(q)(h i) M_q / q!  (Taylor expansion of g under
    the integral; g is entire, the series converges)."""
    with mp.workdps(40):
        M = F.moments_mp(qmax)
        Mw = F.wavelet_moments_mp(qmax)
        s = np.zeros(n)
        d = np.zeros(n)
        hs = mp.mpf(h)
        sg = mp.mpf(sigma)
        for i in range(n):
            u = (hs * i - mp.mpf(x0)) / sg
            g0 = mp.exp(-u * u / 2)
            he_prev, he = mp.mpf(0), mp.mpf(1)       # He_{-1}, He_0
            acc_s = mp.mpf(0)
            acc_d = mp.mpf(0)
            fact = mp.mpf(1)
            for q in range(qmax + 1):
                if q > 0:
                    fact *= q
                der = (-1 / sg) ** q * he * g0        # g^(q)(h i)
                acc_s += hs ** q * der * M[q] / fact
                acc_d += hs ** q * der * Mw[q] / fact
                he_prev, he = he, u * he - q * he_prev
            s[i] = float(mp.sqrt(hs) * acc_s)
            d[i] = float(mp.sqrt(hs) * acc_d)
        return s, d


def test_gauss_projection_has_gaussian_norm():
    h, sigma = 0.4, 1.6
    s, d = gauss_projection_1d(h, sigma, 44 * h / 2, 45)
    assert abs((s @ s + d @ d) / (sigma * math.sqrt(math.pi)) - 1) < 1e-12


# ----------------------------------------------------------------------------
# P5: orthonormal change of basis
# ----------------------------------------------------------------------------

def test_synthesis_is_isometric_and_analysis_inverts_it_1d():
    rng = np.random.default_rng(1)
    for n in (1, 2, 7, 16):
        s, d = rng.standard_normal((2, 3, n))
        sp = W.synthesis_axis(s, d, -1)
        assert sp.shape[-1] == 2 * n + 14
        np.testing.assert_allclose(np.sum(sp ** 2, -1), np.sum(s ** 2 + d ** 2, -1), rtol=1e-14)
        s2, d2 = W.analysis_axis(sp, -1, -7, 0, n)
        np.testing.assert_allclose(s2, s, atol=1e-14)
        np.testing.assert_allclose(d2, d, atol=1e-14)
        # analysis on a wider coarse range gives zeros outside the box
        s3, d3 = W.analysis_axis(sp, -1, -7, -3, n + 6)
        np.testing.assert_allclose(s3[..., 3:3 + n], s, atol=1e-14)
        assert np.max(np.abs(s3[..., :3])) < 1e-14 and np.max(np.abs(d3[..., -3:])) < 1e-14


def test_synthesis_3d_isometric_and_component_order():
    rng = np.random.default_rng(2)
    c8 = rng.standard_normal((8, 3, 4, 5))
    sp = W.synthesis_3d(c8)
    assert sp.shape == (20, 22, 24)
    assert abs(np.sum(sp ** 2) / np.sum(c8 ** 2) - 1) < 1e-14
    back = W.analysis_3d(sp, (-7, -7, -7), (0, 0, 0), (3, 4, 5))
    np.testing.assert_allclose(back, c8, atol=1e-13)
    # component c = a1 + 2 a2 + 4 a3: a single wavelet along x alone (c = 1)
    # synthesises to h-filter profiles along y and z and a g-profile along x
    e = np.zeros((8, 1, 1, 1)); e[1, 0, 0, 0] = 1.0
    sp = W.synthesis_3d(e)
    tab = F.tables()
    expect = np.einsum("k,j,i->kji", tab["h"], tab["h"], tab["g"])
    np.testing.assert_allclose(sp, expect, atol=1e-16)


# ----------------------------------------------------------------------------
# P4: kinetic energy of a Gaussian (closed form 1/(4 sigma^2) per axis)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("ratio,tol", [(4.0, 1e-8), (6.7, 1e-11)])
def test_kinetic_energy_of_gaussian_1d(ratio, tol):
    h = 0.3
    sigma = ratio * h
    n = int(math.ceil(14 * sigma / h)) + 1
    x0 = h * (n - 1) / 2 + 0.123 * h
    s, d = gauss_projection_1d(h, sigma, x0, n)
    sp = W.synthesis_axis(s, d, -1)
    k = (-0.5 * (2 / h) ** 2) * W.kinetic_axis(sp, -1, -7, -7, 2 * n + 14)
    ekin = float(sp @ k) / float(sp @ sp)
    exact = 1.0 / (4 * sigma ** 2)
    assert abs(ekin / exact - 1) < tol, ekin / exact - 1


def _gauss_box(h, sigma, x0, n):
    s, d = gauss_projection_1d(h, sigma, x0, n)
    p = (s, d)
    c8 = np.zeros((8, n, n, n))
    for comp in range(8):
        a1, a2, a3 = comp & 1, (comp >> 1) & 1, (comp >> 2) & 1
        c8[comp] = np.einsum("k,j,i->kji", p[a3], p[a2], p[a1])
    return c8


def _full_box_locreg(n):
    return LR.box_locreg((0, 0, 0), (n, n, n), (0, 0, 0), (n - 1, n - 1, n - 1))


def _compress_full(lr, c8):
    pc = LR.points_from_segments(lr.cseg)
    pf = LR.points_from_segments(lr.fseg)
    fine = np.stack([c8[comp, pf[:, 2], pf[:, 1], pf[:, 0]] for comp in range(1, 8)], axis=1)
    return np.concatenate([c8[0, pc[:, 2], pc[:, 1], pc[:, 0]], fine.reshape(-1)])


def test_local_ham_gaussian_closed_forms_3d():
    """Kinetic 3/(4 sigma^2) and potential <g|V|g> for Gaussian V (product of
    three 1D closed-form integrals) through the full 3D oracle path."""
    h, sigma, n = 0.4, 1.2, 30
    x0 = h * (n - 1) / 2
    c8 = _gauss_box(h, sigma, x0, n)
    lr = _full_box_locreg(n)
    coef = _compress_full(lr, c8)
    norm2 = (sigma * math.sqrt(math.pi)) ** 3
    assert abs(coef @ coef / norm2 - 1) < 1e-10
    # V(r) = A exp(-|r - cv|^2 / (2 w^2)) sampled on the fine grid (p - 14) h/2
    A, w = -1.3, 1.1
    cv = np.array([x0 + 0.31, x0 - 0.2, x0 + 0.05])
    pts = (np.arange(2 * n + 29) - 14) * h / 2
    ex = [np.exp(-(pts - cv[a]) ** 2 / (2 * w * w)) for a in range(3)]
    V = A * np.einsum("k,j,i->kji", ex[2], ex[1], ex[0])
    hp, ek, ep = Hm.apply_local_ham(lr, coef, V, h)
    assert abs(ek / (3 / (4 * sigma ** 2) * norm2) - 1) < 1e-5
    a_, b_ = 1 / sigma ** 2, 1 / (2 * w * w)
    exact = A * np.prod([math.sqrt(math.pi / (a_ + b_)) *
                         math.exp(-a_ * b_ / (a_ + b_) * (x0 - cv[ax]) ** 2) for ax in range(3)])
    assert abs(ep / exact - 1) < 1e-6, ep / exact - 1
    # P11: <phi|H phi> = e_kin + e_pot
    assert abs(coef @ hp - (ek + ep)) < 1e-12 * abs(ek)
    # kinetic-only and potential-only runs add up to the full output
    hk, ek2, _ = Hm.apply_local_ham(lr, coef, V, h, potential=False)
    hv, _, ep2 = Hm.apply_local_ham(lr, coef, V, h, kinetic=False)
    np.testing.assert_allclose(hk + hv, hp, atol=1e-12 * np.max(np.abs(hp)))
    assert ek2 == ek and ep2 == ep


def test_constant_potential_is_identity_on_smooth_functions():
    h, sigma, n = 0.4, 1.2, 30
    c8 = _gauss_box(h, sigma, h * (n - 1) / 2, n)
    lr = _full_box_locreg(n)
    coef = _compress_full(lr, c8)
    V = np.full((2 * n + 29,) * 3, 0.7)
    hv, _, ep = Hm.apply_local_ham(lr, coef, V, h, kinetic=False)
    assert abs(ep / (0.7 * coef @ coef) - 1) < 1e-9
    np.testing.assert_allclose(hv, 0.7 * coef, atol=1e-8 * np.max(np.abs(coef)))


# ----------------------------------------------------------------------------
# P8: brute-force non-separable 3D stencils on tiny boxes
# ----------------------------------------------------------------------------

def _brute_local_h(c8, V, h, ext):
    t = F.tables()
    fil = (np.array(t["h"]), np.array(t["g"]))
    w = np.array(t["magic"])
    a = np.array(t["kinetic"])
    N3, N2, N1 = c8.shape[1:]
    Ns = (2 * N3 + 14, 2 * N2 + 14, 2 * N1 + 14)
    sp = np.zeros(Ns)                                    # m + 7
    for comp in range(8):
        F1, F2, F3 = fil[comp & 1], fil[(comp >> 1) & 1], fil[(comp >> 2) & 1]
        for k3 in range(16):
            for k2 in range(16):
                for k1 in range(16):
                    sp[k3:k3 + 2 * N3:2, k2:k2 + 2 * N2:2, k1:k1 + 2 * N1:2] += \
                        F3[k3] * F2[k2] * F1[k1] * c8[comp]
    Nr = (2 * N3 + 29, 2 * N2 + 29, 2 * N1 + 29)
    f = np.zeros(Nr)                                     # l + 14, l = m + j
    for j3 in range(16):
        for j2 in range(16):
            for j1 in range(16):
                f[j3:j3 + Ns[0], j2:j2 + Ns[1], j1:j1 + Ns[2]] += w[j3] * w[j2] * w[j1] * sp
    g = V * f
    # y on the analysis range m in [-2e-7, 2N+2e+6] (index m + 2e + 7)
    Nb = (2 * N3 + 4 * ext + 14, 2 * N2 + 4 * ext + 14, 2 * N1 + 4 * ext + 14)
    y = np.zeros(Nb)
    off = 2 * ext + 7
    # t_m = sum_j w_j g_{m+j}: g index l+14 with l = m + j
    for j3 in range(16):
        for j2 in range(16):
            for j1 in range(16):
                J = (j3 - 7, j2 - 7, j1 - 7)
                sl_y, sl_g = [], []
                for ax in range(3):
                    # m range such that l = m + J in [-14, 2N+14] and m in range
                    m_lo = max(-off, -14 - J[ax])
                    m_hi = min(Nb[ax] - off - 1, Nr[ax] - 15 - J[ax])
                    sl_y.append(slice(m_lo + off, m_hi + off + 1))
                    sl_g.append(slice(m_lo + J[ax] + 14, m_hi + J[ax] + 15))
                y[tuple(sl_y)] += w[j3] * w[j2] * w[j1] * g[tuple(sl_g)]
    spb = np.zeros(Nb)
    spb[off - 7:off - 7 + Ns[0], off - 7:off - 7 + Ns[1], off - 7:off - 7 + Ns[2]] = sp
    lap = np.zeros(Nb)
    for ax in range(3):
        for li in range(29):
            l = li - 14
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            lo_, hi_ = max(0, -l), min(Nb[ax], Nb[ax] - l)
            dst[ax] = slice(lo_, hi_)
            src[ax] = slice(lo_ + l, hi_ + l)
            lap[tuple(dst)] += a[li] * spb[tuple(src)]
    y += (-0.5 * (2 / h) ** 2) * lap
    No = (N3 + 2 * ext, N2 + 2 * ext, N1 + 2 * ext)
    out = np.zeros((8,) + No)
    for comp in range(8):
        F1, F2, F3 = fil[comp & 1], fil[(comp >> 1) & 1], fil[(comp >> 2) & 1]
        for k3 in range(16):
            for k2 in range(16):
                for k1 in range(16):
                    # i in [-e, N-1+e] reads m = 2i + k at index 2i + k + off
                    out[comp] += F3[k3] * F2[k2] * F1[k1] * y[
                        k3 - 7 - 2 * ext + off:k3 - 7 - 2 * ext + off + 2 * No[0]:2,
                        k2 - 7 - 2 * ext + off:k2 - 7 - 2 * ext + off + 2 * No[1]:2,
                        k1 - 7 - 2 * ext + off:k1 - 7 - 2 * ext + off + 2 * No[2]:2]
    return out


@pytest.mark.parametrize("dims,ext", [((2, 2, 2), 0), ((2, 3, 2), 1)])
def test_separable_oracle_matches_brute_force_3d(dims, ext):
    rng = np.random.default_rng(7)
    n1, n2, n3 = dims
    grid = (n1 + 2 * ext, n2 + 2 * ext, n3 + 2 * ext)
    lo = (ext, ext, ext)
    m = np.ones((n3, n2, n1), bool)
    fm = rng.random((n3, n2, n1)) < 0.6
    om = np.ones((n3 + 2 * ext, n2 + 2 * ext, n1 + 2 * ext), bool)
    lr = LR.Locreg(lo=lo, dims=dims, ext=ext, cseg=LR.segments_from_mask(m, lo),
                   fseg=LR.segments_from_mask(fm, lo), ocseg=LR.segments_from_mask(om, (0, 0, 0)),
                   ofseg=LR.segments_from_mask(om, (0, 0, 0)))
    coef = rng.standard_normal(lr.n_c + 7 * lr.n_f)
    pot = rng.uniform(-1, 0, (2 * grid[2] + 29, 2 * grid[1] + 29, 2 * grid[0] + 29))
    h = 0.5
    hp, ek, ep = Hm.apply_local_ham(lr, coef, pot, h)
    c8 = Hm.uncompress(lr, coef)
    ref = _brute_local_h(c8, Hm.potential_block(lr, pot), h, ext)
    ref_c = Hm.compress_out(lr, ref)
    np.testing.assert_allclose(hp, ref_c, rtol=0, atol=1e-12 * np.max(np.abs(ref_c)))


# ----------------------------------------------------------------------------
# P7: Hermiticity of the localized H when L' covers the operator's full reach
# ----------------------------------------------------------------------------

def test_local_ham_hermitian_at_full_reach():
    h = 0.5
    ext = 26                              # > 15 sqrt(3): L' holds every reached point
    centers = np.array([[20.3, 20.1, 19.7], [21.6, 20.9, 20.2]])
    radii = np.array([1.6, 1.4])
    fine = np.array([0.9, 0.8])
    grid = (82, 82, 82)
    lrs = LR.sphere_locregs(h, grid, centers, radii, fine, ext)
    rng = np.random.default_rng(3)
    coefs = [rng.standard_normal(l.n_c + 7 * l.n_f) for l in lrs]
    pot = np.zeros(tuple(2 * g + 29 for g in grid))
    idx = np.arange(2 * grid[0] + 29)
    sub = slice(60, 110)
    xs = (idx[sub] - 14) * h / 2
    pot[sub, sub, sub] = -1.0 + 0.3 * np.sin(xs)[:, None, None] * np.cos(xs)[None, :, None] \
        + 0.2 * np.cos(0.7 * xs)[None, None, :]
    outs = [Hm.apply_local_ham(l, c, pot, h)[0] for l, c in zip(lrs, coefs)]
    hab = SP.pair_value((lrs[0].cseg, lrs[0].fseg), coefs[0], (lrs[1].ocseg, lrs[1].ofseg), outs[1])
    hba = SP.pair_value((lrs[1].cseg, lrs[1].fseg), coefs[1], (lrs[0].ocseg, lrs[0].ofseg), outs[0])
    scale = math.sqrt(np.dot(outs[0], outs[0]) * np.dot(outs[1], outs[1]))
    assert abs(hab - hba) < 1e-13 * scale, (hab, hba)
    assert abs(hab) > 1e-3 * scale * 1e-3


# ----------------------------------------------------------------------------
# P9: segments and (un)compress
# ----------------------------------------------------------------------------

def test_segments_roundtrip_and_maximal_runs():
    rng = np.random.default_rng(4)
    m = rng.random((5, 6, 9)) < 0.5
    seg = LR.segments_from_mask(m, (3, 4, 5))
    back = LR.mask_from_segments(seg, (3, 4, 5), m.shape)
    assert np.array_equal(back, m)
    key = [(s[3], s[2], s[0]) for s in seg]
    assert key == sorted(key)
    for a, b in zip(seg[:-1], seg[1:]):
        if a[2] == b[2] and a[3] == b[3]:
            assert b[0] > a[1] + 1         # maximal: a gap separates runs in a row


def test_sphere_membership_matches_pointwise_python():
    """Brute force: every grid point tested with Python floats in the stated
    order, (h*i1-X)^2 + (h*i2-Y)^2 + (h*i3-Z)^2 <= R*R."""
    h = 0.45
    grid = (40, 40, 40)
    centers = np.array([[8.1, 8.37, 9.02], [9.5, 7.77, 8.8]])
    radii = np.array([3.1, 2.45])
    fine = np.array([1.4, 1.2])
    lrs = LR.sphere_locregs(h, grid, centers, radii, fine, 3)
    Fset = set()
    for k, l in enumerate(lrs):
        X, Y, Z = centers[k]
        R = radii[k]
        pts = set()
        fpts = set()
        for i3 in range(grid[2]):
            for i2 in range(grid[1]):
                for i1 in range(grid[0]):
                    dx = h * i1 - X; dy = h * i2 - Y; dz = h * i3 - Z
                    d2 = (dx * dx + dy * dy) + dz * dz
                    if d2 <= R * R:
                        pts.add((i1, i2, i3))
                        if d2 <= fine[k] * fine[k]:
                            fpts.add((i1, i2, i3))
        assert set(map(tuple, LR.points_from_segments(l.cseg))) == pts
        assert set(map(tuple, LR.points_from_segments(l.fseg))) == fpts
        Fset |= fpts
    for k, l in enumerate(lrs):
        X, Y, Z = centers[k]
        Rp = radii[k] + 3 * h
        lo = [l.lo[a] - 3 for a in range(3)]
        hi = [l.lo[a] + l.dims[a] - 1 + 3 for a in range(3)]
        opts = set()
        for i3 in range(lo[2], hi[2] + 1):
            for i2 in range(lo[1], hi[1] + 1):
                for i1 in range(lo[0], hi[0] + 1):
                    dx = h * i1 - X; dy = h * i2 - Y; dz = h * i3 - Z
                    if (dx * dx + dy * dy) + dz * dz <= Rp * Rp:
                        opts.add((i1, i2, i3))
        assert set(map(tuple, LR.points_from_segments(l.ocseg))) == opts
        assert set(map(tuple, LR.points_from_segments(l.ofseg))) == opts & Fset


def test_uncompress_compress_identity_on_pattern():
    # one support function: the union F of fine sets is its own fine set,
    # so with ext = 0 the output pattern equals the input pattern
    g = inputs.geometry("batch1k", nsf=1)
    lrs = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, 0)
    l = lrs[0]
    assert np.array_equal(l.ocseg, l.cseg) and np.array_equal(l.ofseg, l.fseg)
    coef = np.random.default_rng(0).standard_normal(l.n_c + 7 * l.n_f)
    assert np.array_equal(Hm.compress_out(l, Hm.uncompress(l, coef)), coef)


# ----------------------------------------------------------------------------
# P10: S and H values against a dictionary-based scalar product
# ----------------------------------------------------------------------------

def _dict_of(seg_c, seg_f, coef):
    pc = LR.points_from_segments(seg_c)
    pf = LR.points_from_segments(seg_f)
    d = {}
    for i, p in enumerate(map(tuple, pc)):
        d[(p, 0)] = coef[i]
    nc = len(pc)
    for i, p in enumerate(map(tuple, pf)):          # [d: n_f][7]
        for comp in range(1, 8):
            d[(p, comp)] = coef[nc + 7 * i + (comp - 1)]
    return d


def test_sparse_matrices_against_dictionary_products():
    g = inputs.geometry("batch1k", nsf=6)
    g.centers[:] = g.centers[0] + np.random.default_rng(9).uniform(-4, 4, (6, 3))
    lrs = LR.sphere_locregs(g.h, g.grid_n, g.centers, np.full(6, 2.5), np.full(6, 1.2), 2)
    rng = np.random.default_rng(10)
    bra = [rng.standard_normal(l.n_c + 7 * l.n_f) for l in lrs]
    ket = [rng.standard_normal(l.on_c + 7 * l.on_f) for l in lrs]
    for out in (False, True):
        rowptr, col, val = SP.matrix(lrs, bra, ket if out else bra, out)
        n = 0
        for a in range(6):
            da = _dict_of(lrs[a].cseg, lrs[a].fseg, bra[a])
            for b in range(6):
                lb = lrs[b]
                db = _dict_of(lb.ocseg, lb.ofseg, ket[b]) if out else _dict_of(lb.cseg, lb.fseg, bra[b])
                common_c = {k[0] for k in da if k[1] == 0} & {k[0] for k in db if k[1] == 0}
                cols = list(col[rowptr[a]:rowptr[a + 1]])
                assert (b in cols) == bool(common_c)
                if common_c:
                    ref = sum(v * db[k] for k, v in da.items() if k in db)
                    got = val[rowptr[a] + cols.index(b)]
                    assert abs(got - ref) < 1e-12 * (1 + abs(ref))
                    n += 1
        assert n > 6
    rowptr, col, val = SP.matrix(lrs, bra, bra, False)
    S = np.zeros((6, 6))
    for a in range(6):
        for j in range(rowptr[a], rowptr[a + 1]):
            S[a, col[j]] = val[j]
    np.testing.assert_allclose(S, S.T, atol=1e-13)
    for a in range(6):
        assert abs(S[a, a] - bra[a] @ bra[a]) < 1e-12


def _layout(cseg, fseg):
    """(component, point) of each compressed coefficient, in storage order:
    coarse points (scaling), then each fine point's seven wavelets."""
    return ([(0, p) for p in LR.points_from_segments(cseg)] +
            [(c, p) for p in LR.points_from_segments(fseg) for c in range(1, 8)])


# P12: the update step's projection P_L is a pointwise restriction
def test_update_restriction_matches_pointwise_dictionary():
    from oracle import update as U
    rng = np.random.default_rng(17)
    g = inputs.geometry("batch1k", nsf=3)
    lrs = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii * 0.5, g.fine_radii * 0.5, 3)
    for lr in lrs:
        out = rng.standard_normal(lr.on_c + 7 * lr.on_f)
        # dictionary: (component, point) -> value of the output-layout vector
        d = {}
        k = 0
        for comp, p in _layout(lr.ocseg, lr.ofseg):
            d[(comp, tuple(int(v) for v in p))] = out[k]
            k += 1
        want = []
        for comp, p in _layout(lr.cseg, lr.fseg):
            want.append(d[(comp, tuple(int(v) for v in p))])
        got = U.restrict_to_input(lr, out)
        assert np.array_equal(got, np.array(want))
        psi = rng.standard_normal(lr.n_c + 7 * lr.n_f)
        assert np.array_equal(U.update(lr, psi, out, 0.7, 0.0), psi)
        # with H phi = c phi on the pattern the step leaves phi unchanged
        emb = np.zeros_like(out)
        k = 0
        inv = {}
        for comp, p in _layout(lr.cseg, lr.fseg):
            inv[(comp, tuple(int(v) for v in p))] = psi[k]
            k += 1
        k = 0
        for comp, p in _layout(lr.ocseg, lr.ofseg):
            emb[k] = 2.5 * inv.get((comp, tuple(int(v) for v in p)), 0.0)
            k += 1
        assert np.allclose(U.update(lr, psi, emb, 2.5, 0.01), psi, rtol=0, atol=1e-15)


# P13: the confining potential a |r - R|^4 on a Gaussian: <r^4> = 15 s^4 / 4
def test_confinement_energy_of_a_gaussian():
    h, sigma, n = 0.4, 1.2, 30
    x0 = h * (n - 1) / 2
    c8 = _gauss_box(h, sigma, x0, n)
    lr = _full_box_locreg(n)
    coef = _compress_full(lr, c8)
    norm2 = (sigma * math.sqrt(math.pi)) ** 3
    a = 0.037
    zero = np.zeros((2 * n + 29,) * 3)
    _, _, ep = Hm.apply_local_ham(lr, coef, zero, h, kinetic=False, conf=a,
                                  center=(x0, x0, x0))
    exact = a * 15.0 * sigma ** 4 / 4.0 * norm2
    assert abs(ep / exact - 1) < 1e-8, ep / exact - 1
    # an off-centre confinement adds the shift terms of (r - d)^4 averaged
    d = np.array([0.3, -0.2, 0.1])
    _, _, ep2 = Hm.apply_local_ham(lr, coef, zero, h, kinetic=False, conf=a,
                                   center=tuple(x0 + d))
    v = sigma ** 2 / 2                      # per-axis variance of |g|^2
    dd = float(d @ d)
    # E|x - d|^4 for an isotropic normal: 15 v^2 + 10 v |d|^2 + |d|^4
    exact2 = a * (15 * v * v + 10 * v * dd + dd * dd) * norm2
    assert abs(ep2 / exact2 - 1) < 1e-8, ep2 / exact2 - 1


# P14: the preconditioner's operator is symmetric positive definite, and its
# conjugate-gradient solve reaches the dense direct solution
def test_preconditioner_against_a_dense_solve():
    from oracle import precond as PC
    h = 0.5
    lo, dims = (3, 3, 3), (6, 6, 6)
    m = np.ones((6, 6, 6), bool)
    fm = np.zeros_like(m)
    fm[2:4, 2:4, 2:4] = True
    ext = 2
    olo = [v - ext for v in lo]
    om = np.ones((10, 10, 10), bool)
    ofm = np.zeros_like(om)
    ofm[ext + 2:ext + 4, ext + 2:ext + 4, ext + 2:ext + 4] = True
    lr = LR.Locreg(lo=lo, dims=dims, ext=ext, cseg=LR.segments_from_mask(m, lo),
                   fseg=LR.segments_from_mask(fm, lo), ocseg=LR.segments_from_mask(om, olo),
                   ofseg=LR.segments_from_mask(ofm, olo), center=(3.2, 3.1, 2.9))
    n = lr.n_c + 7 * lr.n_f
    conf, eps = 0.02, -0.7
    A = np.stack([PC.apply_operator(lr, np.eye(n)[i], h, conf, eps) for i in range(n)], axis=1)
    assert np.max(np.abs(A - A.T)) < 1e-12 * np.max(np.abs(A))
    w = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert w[0] > 0.69                       # T + C >= 0, shifted by 0.7
    g = np.random.default_rng(3).standard_normal(n)
    direct = np.linalg.solve(A, -g)
    x = PC.precondition(lr, g, h, conf, eps, niter=n)
    assert np.linalg.norm(x - direct) < 1e-8 * np.linalg.norm(direct)
    # a positive eps is taken as 0: the operator is then T + C
    A0 = np.stack([PC.apply_operator(lr, np.eye(n)[i], h, conf, 0.4) for i in range(n)], axis=1)
    A1 = np.stack([PC.apply_operator(lr, np.eye(n)[i], h, conf, 0.0) for i in range(n)], axis=1)
    assert np.array_equal(A0, A1)


def test_sphere_set_coarse_sets_match_segments():
    """SphereSet.coarse_set (the masks the sampled full-size tests intersect
    to find pattern rows) equals the locreg's own segment lists, input and
    output, and one function's locreg does not depend on which others are
    built."""
    import inputs
    g = inputs.geometry("batch1k", nsf=6)
    S = LR.SphereSet(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
    full = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
    for k in (4, 1):
        l = S.locreg(k)
        for a, b in ((l.cseg, full[k].cseg), (l.ocseg, full[k].ocseg), (l.ofseg, full[k].ofseg)):
            assert np.array_equal(a, b)
        for out, seg in ((False, l.cseg), (True, l.ocseg)):
            m, lo = S.coarse_set(k, out)
            assert np.array_equal(LR.mask_from_segments(seg, lo, m.shape), m)
