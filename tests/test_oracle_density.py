"""Pins of the density oracle (paper Sec. II, Eqs. (expansion) and (density)).

* Sum rule: the fine-box values of a function add up to 2 sqrt(2) times the
  sum of its coarse scaling coefficients (the low-pass synthesis filter sums
  to sqrt(2) per axis, the wavelet filter to zero, the magic filter to one),
  which holds only if the fine box holds every filter tail.
* Orbital form: with K = sum_i f_i c_i c_i^T, rho = sum_i f_i Psi_i(r)^2
  where Psi_i = sum_a c_i^a phi_a is synthesized once on the whole grid, so
  the per-function placement at global fine index 2 lo + l + 14 and the
  contraction with K are checked against an independent path.
"""
import numpy as np
import pytest

from oracle import density as D
from oracle import hamiltonian as Hm
from oracle import locreg as LR
from oracle import wavelet as W

GRID = (15, 14, 13)
H = 0.5


def _case(seed, nsf=4):
    rng = np.random.default_rng(seed)
    centers = rng.uniform(2.2, 4.3, (nsf, 3))
    radii = rng.uniform(1.4, 2.1, nsf)
    lrs = LR.sphere_locregs(H, GRID, centers, radii, np.minimum(1.0, radii), 0)
    coefs = [rng.standard_normal(lr.n_c + 7 * lr.n_f) for lr in lrs]
    return lrs, coefs, rng


@pytest.mark.parametrize("seed", [1, 2])
def test_fine_values_sum_rule(seed):
    lrs, coefs, _ = _case(seed)
    for lr, c in zip(lrs, coefs):
        f = D.fine_values(lr, c)
        assert f.shape == D.fine_box_shape(lr)
        want = 2.0 * np.sqrt(2.0) * np.sum(c[:lr.n_c])
        assert abs(np.sum(f) - want) <= 1e-12 * np.sum(np.abs(f))


def _global_fine(lrs, coefs, weights):
    """sum_a w_a phi_a synthesized on the whole coarse grid (origin 0)."""
    g = np.zeros((8, GRID[2], GRID[1], GRID[0]))
    for lr, c, w in zip(lrs, coefs, weights):
        box = Hm.uncompress(lr, c)
        lo, n = lr.lo, lr.dims
        g[:, lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]] += w * box
    sp = W.synthesis_3d(g)
    shape = (2 * GRID[2] + 29, 2 * GRID[1] + 29, 2 * GRID[0] + 29)
    return W.magic_3d(sp, (-7, -7, -7), (-14, -14, -14), shape)


@pytest.mark.parametrize("seed", [3, 4])
def test_density_equals_orbital_form(seed):
    lrs, coefs, rng = _case(seed)
    nsf, norb = len(lrs), 3
    c = rng.standard_normal((norb, nsf))
    f = rng.uniform(0.2, 2.0, norb)
    K = sum(f[i] * np.outer(c[i], c[i]) for i in range(norb))
    want = sum(f[i] * _global_fine(lrs, coefs, c[i]) ** 2 for i in range(norb))
    got = D.density(lrs, coefs, K, GRID)
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    # the same kernel in CSR form
    rowptr = np.arange(nsf + 1) * nsf
    col = np.tile(np.arange(nsf), nsf)
    got2 = D.density(lrs, coefs, (rowptr, col, K.ravel()), GRID)
    assert np.array_equal(got, got2)
    assert np.min(got) >= -1e-12 * np.max(got)     # K positive semidefinite
