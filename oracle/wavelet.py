"""Dense-box wavelet operators in FP64 (TEST INFRASTRUCTURE ONLY: oracle).

Paper, Sec. III.B: the local Hamiltonian acts through convolutions; Eq. (Phi)
of Sec. II.B gives the two-level expansion (one scaling function on coarse
points, plus seven wavelets on fine points) that these operators transform.

Index conventions (readings listed in the design notes):
  * A box of N coarse points per axis has local coarse indices i = 0..N-1.
  * Synthesis to the h/2 scaling level gives m = -7..2N+6 (N_s = 2N+14).
  * The magic filter gives fine real-space points l = -14..2N+14 (N_r = 2N+29);
    local l sits at global fine index 2*lo + l + 14.
  * Component c = a1 + 2*a2 + 4*a3 of the 8-component coarse box, a_d = 1
    meaning a wavelet (filter g) along axis d; axis 1 = x is the fastest.
  * Arrays are stored [..., z, y, x]; axis -1 = x, -2 = y, -3 = z.

Every 1D operator is the plain definition written as a loop over filter taps,
each tap a shifted-slice multiply-add; nothing is blocked or fused.
"""
from __future__ import annotations

import numpy as np

from . import filters as _filters

LO, HI = _filters.LO, _filters.HI          # -7, 8
KLO, KHI = _filters.KLO, _filters.KHI      # -14, 14


def _tab():
    t = _filters.tables()
    return (np.array(t["h"]), np.array(t["g"]), np.array(t["magic"]),
            np.array(t["kinetic"]))


def correlate_axis(x, axis, x_lo, out_lo, out_n, taps_lo, taps):
    """out[m] = sum_j taps[j - taps_lo] * x[m + j], m in [out_lo, out_lo + out_n).

    x holds indices [x_lo, x_lo + x.shape[axis]) along `axis` and is zero
    outside them.  Plain tap loop."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    nx = x.shape[-1]
    out = np.zeros(x.shape[:-1] + (out_n,), dtype=np.float64)
    for t, w in enumerate(taps):
        j = taps_lo + t
        # output m such that x_lo <= m + j < x_lo + nx
        m_begin = max(out_lo, x_lo - j)
        m_end = min(out_lo + out_n, x_lo + nx - j)
        if m_end <= m_begin:
            continue
        out[..., m_begin - out_lo:m_end - out_lo] += w * x[..., m_begin + j - x_lo:m_end + j - x_lo]
    return np.moveaxis(out, -1, axis)


def synthesis_axis(s, d, axis):
    """Coarse (s_i, d_i), i = 0..N-1  ->  h/2 scaling coefficients
    s'_m = sum_i h_{m-2i} s_i + g_{m-2i} d_i,  m = -7..2N+6.
    (Change of basis phi^h_i = sum_k h_k phi^{h/2}_{2i+k}, psi^h_i likewise with g.)"""
    h, g, _, _ = _tab()
    s = np.moveaxis(np.asarray(s, np.float64), axis, -1)
    d = np.moveaxis(np.asarray(d, np.float64), axis, -1)
    n = s.shape[-1]
    out = np.zeros(s.shape[:-1] + (2 * n + 14,), np.float64)
    for t in range(16):
        k = LO + t
        # m = 2i + k, stored at m + 7
        start = k + 7
        out[..., start:start + 2 * n:2] += h[t] * s + g[t] * d
    return np.moveaxis(out, -1, axis)


def analysis_axis(y, axis, y_lo, i_lo, i_n):
    """h/2 coefficients y_m (indices [y_lo, y_lo + len)) -> coarse pairs
    s_i = sum_k h_k y_{2i+k},  d_i = sum_k g_k y_{2i+k},  i in [i_lo, i_lo + i_n).
    The adjoint of synthesis_axis (orthonormal basis)."""
    h, g, _, _ = _tab()
    y = np.moveaxis(np.asarray(y, np.float64), axis, -1)
    ny = y.shape[-1]
    # zero-padded copy covering every 2i+k the outputs touch
    need_lo = 2 * i_lo + LO
    need_n = 2 * i_n + 14
    ypad = np.zeros(y.shape[:-1] + (need_n,), np.float64)
    b = max(need_lo, y_lo)
    e = min(need_lo + need_n, y_lo + ny)
    if e > b:
        ypad[..., b - need_lo:e - need_lo] = y[..., b - y_lo:e - y_lo]
    s = np.zeros(y.shape[:-1] + (i_n,), np.float64)
    d = np.zeros_like(s)
    for t in range(16):
        # m = 2i + k sits at ypad position 2(i - i_lo) + t
        sl = ypad[..., t:t + 2 * i_n:2]
        s += h[t] * sl
        d += g[t] * sl
    return np.moveaxis(s, -1, axis), np.moveaxis(d, -1, axis)


def magic_axis(sp, axis, sp_lo, out_lo, out_n):
    """Point values f_l = sum_m w_{l-m} s'_m = sum_j w_j s'_{l-j}."""
    _, _, w, _ = _tab()
    # correlation form: taps at offsets -j for j = -7..8, i.e. offsets -8..7
    return correlate_axis(sp, axis, sp_lo, out_lo, out_n, -HI, w[::-1])


def magic_t_axis(f, axis, f_lo, out_lo, out_n):
    """Transposed magic filter t_m = sum_l w_{l-m} f_l = sum_j w_j f_{m+j}."""
    _, _, w, _ = _tab()
    return correlate_axis(f, axis, f_lo, out_lo, out_n, LO, w)


def kinetic_axis(sp, axis, sp_lo, out_lo, out_n):
    """Second-derivative filter along one axis: k_m = sum_l a_l s'_{m+l}
    (unit spacing; the caller applies -1/2 (2/h)^2)."""
    _, _, _, a = _tab()
    return correlate_axis(sp, axis, sp_lo, out_lo, out_n, KLO, a)


# ----------------------------------------------------------------------------
# 3D operators on 8-component coarse boxes  (array shape (8, N3, N2, N1))
# ----------------------------------------------------------------------------

def synthesis_3d(c8):
    """(8, N3, N2, N1) two-level coefficients -> h/2 scaling coefficients of
    shape (2N3+14, 2N2+14, 2N1+14), origin -7 on every axis."""
    c8 = np.asarray(c8, np.float64)
    assert c8.shape[0] == 8
    # x: component pairs differ in a1 (bit 0)
    sx = [synthesis_axis(c8[2 * q], c8[2 * q + 1], -1) for q in range(4)]   # q = a2 + 2 a3
    sy = [synthesis_axis(sx[2 * r], sx[2 * r + 1], -2) for r in range(2)]   # r = a3
    return synthesis_axis(sy[0], sy[1], -3)


def analysis_3d(y, y_lo, i_lo, i_n):
    """h/2 coefficients y (origin y_lo = (lo_z, lo_y, lo_x) per axis) ->
    (8, n3, n2, n1) two-level coefficients on coarse indices
    [i_lo[a], i_lo[a] + i_n[a]) per axis (given z, y, x)."""
    z0, z1 = analysis_axis(y, -3, y_lo[0], i_lo[0], i_n[0])
    out = [None] * 8
    for a3, yz in enumerate((z0, z1)):
        y0, y1 = analysis_axis(yz, -2, y_lo[1], i_lo[1], i_n[1])
        for a2, yy in enumerate((y0, y1)):
            x0, x1 = analysis_axis(yy, -1, y_lo[2], i_lo[2], i_n[2])
            out[0 + 2 * a2 + 4 * a3] = x0
            out[1 + 2 * a2 + 4 * a3] = x1
    return np.stack(out)


def magic_3d(sp, sp_lo, out_lo, out_n):
    """Separable magic filter along x, y, z (per-axis origins/lengths given z, y, x)."""
    f = magic_axis(sp, -1, sp_lo[2], out_lo[2], out_n[2])
    f = magic_axis(f, -2, sp_lo[1], out_lo[1], out_n[1])
    return magic_axis(f, -3, sp_lo[0], out_lo[0], out_n[0])


def magic_t_3d(f, f_lo, out_lo, out_n):
    t = magic_t_axis(f, -1, f_lo[2], out_lo[2], out_n[2])
    t = magic_t_axis(t, -2, f_lo[1], out_lo[1], out_n[1])
    return magic_t_axis(t, -3, f_lo[0], out_lo[0], out_n[0])


def embed(x, x_lo, out_lo, out_n):
    """Zero-padded copy of x (origins x_lo) onto the box [out_lo, out_lo+out_n)."""
    out = np.zeros(tuple(out_n), np.float64)
    src = []
    dst = []
    for a in range(3):
        b = max(x_lo[a], out_lo[a])
        e = min(x_lo[a] + x.shape[a], out_lo[a] + out_n[a])
        if e <= b:
            return out
        src.append(slice(b - x_lo[a], e - x_lo[a]))
        dst.append(slice(b - out_lo[a], e - out_lo[a]))
    out[tuple(dst)] = x[tuple(src)]
    return out


def laplacian_sum_3d(sp_on_box, lo):
    """sum over axes of the unit-spacing second-derivative filter, on a box
    whose input is already embedded (zero outside its support)."""
    n = sp_on_box.shape
    return (kinetic_axis(sp_on_box, -1, lo[2], lo[2], n[2])
            + kinetic_axis(sp_on_box, -2, lo[1], lo[1], n[1])
            + kinetic_axis(sp_on_box, -3, lo[0], lo[0], n[0]))
