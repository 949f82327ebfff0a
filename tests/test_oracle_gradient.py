"""Pins of the gradient oracle (Eq. (gradient), Sec. IV.A; localization
Sec. III.A), none of which reuses the oracle's own formulas:

* the vector part against a brute force on one dense box holding every
  function (placement of coarse and fine points, the seven wavelets, the
  restriction to L^a, the two terms and their signs);
* for orthonormal functions, a symmetric H and a kernel that commutes with
  it, the Lagrange term removes exactly the part of sum_d K_ad H|phi_d>
  inside the span of the functions: the gradient is orthogonal to all of
  them and equals sum_d K_ad of the part of H|phi_d> outside the span;
* the first-order Taylor S^-1 against the exact inverse, to second order in
  the deviation from orthonormality;
* the truncated products against plain loops over the pattern.
"""
import numpy as np

import inputs
from oracle import gradient as G
from oracle import locreg as LR


def _pts(seg):
    return [tuple(int(v) for v in p) for p in LR.points_from_segments(seg)]


def _sym(rng, n, scale=1.0):
    a = rng.standard_normal((n, n)) * scale
    return 0.5 * (a + a.T)


def _spheres(nsf=5, seed=3):
    g = inputs.geometry("batch1k", nsf=nsf, seed_offset=seed)
    rng = np.random.default_rng(seed)
    g.centers[:] = g.centers.mean(0) + rng.uniform(-3.0, 3.0, (nsf, 3))
    g.radii[:] = rng.uniform(2.2, 3.0, nsf)
    g.fine_radii[:] = 1.4
    return LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, 3)


def test_vector_part_against_dense_global_box():
    lrs = _spheres()
    n = len(lrs)
    rng = np.random.default_rng(1)
    psi = [rng.standard_normal(l.n_c + 7 * l.n_f) for l in lrs]
    hpsi = [rng.standard_normal(l.on_c + 7 * l.on_f) for l in lrs]
    mask = rng.random((n, n)) < 0.7
    np.fill_diagonal(mask, True)
    A = rng.standard_normal((n, n)) * mask
    M = rng.standard_normal((n, n)) * mask
    got = G.gradient(lrs, psi, hpsi, A, M, mask)
    # one dense box [8][z][y][x] over every function's output box
    lo = np.min([[l.lo[a] - l.ext for a in range(3)] for l in lrs], axis=0)
    hi = np.max([[l.lo[a] + l.dims[a] + l.ext for a in range(3)] for l in lrs], axis=0)
    shape = (8, hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])

    def dense(cseg, fseg, coef):
        box = np.zeros(shape)
        pc, pf = _pts(cseg), _pts(fseg)
        for k, (x, y, z) in enumerate(pc):
            box[0, z - lo[2], y - lo[1], x - lo[0]] = coef[k]
        for k, (x, y, z) in enumerate(pf):
            for comp in range(1, 8):
                box[comp, z - lo[2], y - lo[1], x - lo[0]] = coef[len(pc) + 7 * k + comp - 1]
        return box
    phis = [dense(l.cseg, l.fseg, psi[k]) for k, l in enumerate(lrs)]
    hphis = [dense(l.ocseg, l.ofseg, hpsi[k]) for k, l in enumerate(lrs)]
    for a, la in enumerate(lrs):
        box = np.zeros(shape)
        for d in range(n):
            if mask[a, d]:
                box += A[a, d] * hphis[d] - M[a, d] * phis[d]
        pc, pf = _pts(la.cseg), _pts(la.fseg)
        want = [box[0, z - lo[2], y - lo[1], x - lo[0]] for (x, y, z) in pc]
        for (x, y, z) in pf:
            want += [box[comp, z - lo[2], y - lo[1], x - lo[0]] for comp in range(1, 8)]
        assert np.max(np.abs(got[a] - np.array(want))) < 1e-13, a


def test_gradient_orthogonal_to_the_functions_when_kernel_commutes():
    """All functions on one box pattern (L^a is then the identity on them),
    orthonormal (S = I, where the Taylor S^-1 is exact), H = Phi^T V
    symmetric, K = f(H)."""
    lr = LR.box_locreg((0, 0, 0), (6, 5, 4), (1, 1, 1), (3, 3, 2))
    dim = lr.n_c + 7 * lr.n_f
    n = 6
    rng = np.random.default_rng(2)
    phi, _ = np.linalg.qr(rng.standard_normal((dim, n)))       # columns orthonormal
    C = _sym(rng, n)
    w = rng.standard_normal((dim, n))
    wperp = w - phi @ (phi.T @ w)                              # outside the span
    V = phi @ C + wperp                                        # "H phi_d" = column d
    lam, U = np.linalg.eigh(C)
    K = (U * (1.0 / (1.0 + np.exp(3.0 * lam)))) @ U.T          # commutes with C
    S = phi.T @ phi
    H = phi.T @ V
    assert np.max(np.abs(S - np.eye(n))) < 1e-13 and np.max(np.abs(H - H.T)) < 1e-13
    mask = np.ones((n, n), bool)
    A, M = G.coefficient_matrices(S, H, K, mask)
    g = G.gradient([lr] * n, [phi[:, k] for k in range(n)], [V[:, k] for k in range(n)], A, M,
                   mask)
    g = np.stack(g, axis=1)
    assert np.max(np.abs(phi.T @ g)) < 1e-12
    assert np.max(np.abs(g - wperp @ K)) < 1e-12               # K symmetric: sum_d K_ad w_d


def test_taylor_inverse_to_second_order():
    rng = np.random.default_rng(4)
    n = 8
    H, K = _sym(rng, n), _sym(rng, n)
    mask = np.ones((n, n), bool)
    E = _sym(rng, n)
    errs = []
    for eps in (1e-2, 5e-3):
        S = np.eye(n) + eps * E
        A, M = G.coefficient_matrices(S, H, K, mask)
        lam = H @ K @ S
        exact = 0.5 * np.linalg.inv(S) @ (lam + lam.T)
        assert np.max(np.abs(A - S @ K)) < 1e-13
        errs.append(np.max(np.abs(M - exact)))
    # second order: halving eps quarters the error
    assert errs[0] < 50 * 1e-4 and 3.0 < errs[0] / errs[1] < 5.0


def test_truncated_products_against_loops_over_the_pattern():
    rng = np.random.default_rng(5)
    n = 12
    i = np.arange(n)
    mask = np.abs(i[:, None] - i[None, :]) <= 2
    S = (np.eye(n) + _sym(rng, n, 0.05)) * mask
    H = rng.standard_normal((n, n)) * mask                     # not symmetric
    K = _sym(rng, n) * mask
    A, M = G.coefficient_matrices(S, H, K, mask)
    P = [(a, b) for a in range(n) for b in range(n) if mask[a, b]]
    row = {a: [b for b in range(n) if mask[a, b]] for a in range(n)}
    X, lam, A2, M2 = {}, {}, {}, {}
    for a, c in P:
        X[a, c] = sum(H[a, d] * K[d, c] for d in row[a] if mask[d, c])
        A2[a, c] = sum(S[a, b] * K[b, c] for b in row[a] if mask[b, c])
    for a, b in P:
        lam[a, b] = sum(X[a, c] * S[c, b] for c in row[a] if mask[c, b])
    for a, b in P:
        M2[a, b] = 0.5 * sum(((2.0 if a == c else 0.0) - S[a, c]) * (lam[c, b] + lam[b, c])
                             for c in row[a] if mask[c, b])
    for a in range(n):
        for b in range(n):
            if mask[a, b]:
                assert abs(A[a, b] - A2[a, b]) < 1e-13 and abs(M[a, b] - M2[a, b]) < 1e-13
            else:
                assert A[a, b] == 0.0 and M[a, b] == 0.0
