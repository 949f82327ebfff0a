"""Fermi operator expansion (paper Sec. IV.B, App. B) through the C ABI
against the oracle, on S and H computed by the oracle (the same values feed
both sides).  Both sides run the same steps in double, with sums in other
orders, coefficients from 16384 (oracle) and max(8 npl, 2048) (library)
quadrature nodes, and their own bisections.  The tolerances follow from the
error terms (_tolerances below):
  * bisection: both stop at a width of 1e-13 (|lo| + |hi|), lo and hi the
    spectral bounds widened by 20 delta, so |d mu| <= 2e-13 (|lo| + |hi|);
    then |dK| <= |d mu| max|f'| |S^-1/2|^2, with max|f'| = 1 / (delta
    sqrt(pi)) and |S^-1/2| <= 1.5 for the overlaps here;
  * Chebyshev recursion in [-1, 1]: rounding grows at most linearly with the
    degree, npl eps sum_i |c_i| < 1e-12;
  * quadrature of the coefficients: the Fermi function's Chebyshev series
    has decayed below 1e-16 long before the 2048th node on these spectra.
E_BS: relative 1e-10 (a trace of K H~ plus tau Tr K S, |dK| scaled).
Measured on the GPU: K <= 4.2e-14 of its largest entry, mu <= 7.8e-14,
E_BS <= 2.9e-13 relative."""
import numpy as np
import pytest

from oracle import foe as F
from oracle import locreg as LR
from oracle import sparse as SP
from tests.abi_helpers import to_abi
from tests.test_gpu_parity import _print, _sphere_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1401_7441_amd as W


@pytest.fixture(scope="module")
def system():
    case = _sphere_case(nsf=10, seed_shift=5)
    n = len(case.lrs)
    ohs = [case.oracle(k)[0] for k in range(n)]
    s = SP.matrix(case.lrs, case.coefs, case.coefs, False)
    h = SP.matrix(case.lrs, case.coefs, ohs, True)
    return case, s, h


def _tolerances(bounds, delta):
    """(|dK| / max|K|, |d mu|) allowed, from the bisection width and the
    recursion's rounding (see the module docstring)."""
    lo, hi = bounds[0] - 20.0 * delta, bounds[1] + 20.0 * delta
    dmu = 2e-13 * max(1.0, abs(lo) + abs(hi)) + 1e-12
    dk = dmu / (delta * np.sqrt(np.pi)) * 2.25 + 1e-12
    return dk, dmu


def _dense(n, rp, cl, vv):
    A = np.zeros((n, n))
    for a in range(n):
        A[a, cl[rp[a]:rp[a + 1]]] = vv[rp[a]:rp[a + 1]]
    return A


@pytest.mark.parametrize("bounds", ["gershgorin", "given"])
def test_foe_against_oracle(system, bounds):
    _print(f"case: FOE, {bounds} bounds")
    case, (srp, scl, sv), (hrp, hcl, hv) = system
    n = len(case.lrs)
    ctx = W.Context(case.g.h, case.g.grid_n)
    plan = W.Plan(ctx, case.rec, case.segs)
    psi = torch.tensor(case.psi, dtype=torch.float64, device="cuda")
    rowptr, col, _ = W.sparse_overlap(plan, psi, psi, False)
    assert np.array_equal(rowptr.cpu().numpy(), srp) and np.array_equal(col.cpu().numpy(), scl)
    S, H = _dense(n, srp, scl, sv), _dense(n, hrp, hcl, hv)
    mask = _dense(n, srp, scl, np.ones(len(scl))) > 0
    npl, delta, nocc = 90, 0.25, 0.5 * n
    emin, emax = (None, None)
    if bounds == "given":
        lam = np.linalg.eigvalsh(0.5 * (H + H.T) * mask)
        emin, emax = float(lam[0] - 0.5), float(lam[-1] + 0.5)
    K, mu, ebs, bnd = F.foe(S, H, mask, npl, delta, nocc, emin, emax)
    ktol, mtol = _tolerances(bnd, delta)
    kv, gmu, gebs = W.foe(plan, torch.tensor(sv, device="cuda"), torch.tensor(hv, device="cuda"),
                          npl, delta, nocc, emin or 0.0, emax or 0.0)
    got = kv.cpu().numpy()
    want = np.array([K[a, scl[q]] for a in range(n) for q in range(srp[a], srp[a + 1])])
    _print(f"  K err {np.max(np.abs(got - want)):.2e} of max |K| {np.max(np.abs(want)):.2f}, "
           f"mu err {abs(gmu - mu):.2e}, E_BS err {abs(gebs - ebs):.2e}")
    assert np.max(np.abs(got - want)) <= ktol * np.max(np.abs(want))
    assert abs(gmu - mu) <= mtol
    assert abs(gebs - ebs) <= 1e-10 * max(1.0, abs(ebs))
    # bitwise reproducible, and the same bits when the Chebyshev matrices are
    # formed twice (smaller scratch) instead of kept
    for keep in (True, False):
        kv2, mu2, ebs2 = W.foe(plan, torch.tensor(sv, device="cuda"),
                               torch.tensor(hv, device="cuda"), npl, delta, nocc, emin or 0.0,
                               emax or 0.0, keep=keep)
        assert np.array_equal(kv2.cpu().numpy(), got) and mu2 == gmu and ebs2 == gebs, keep


def _cluster_plan(m):
    """Three clusters of m identical boxes (11 x 7 x 7 coarse points, output =
    input) at x = 0, 8 and 16: boxes of clusters c and c' share points iff
    |c - c'| <= 1, so the overlap pattern is known in closed form.  Rows of
    the outer clusters miss the columns of the far cluster that rows of the
    middle one hold."""
    lrs = []
    for c in range(3):
        for _ in range(m):
            lrs.append(LR.box_locreg((8 * c, 0, 0), (11, 7, 7), (8 * c + 3, 2, 2),
                                     (8 * c + 6, 4, 4)))
    ctx = W.Context(0.45, (32, 16, 16))
    rec, segs = to_abi(lrs)
    plan = W.Plan(ctx, rec, segs)
    cl = np.repeat(np.arange(3), m)
    mask = np.abs(cl[:, None] - cl[None, :]) <= 1
    return ctx, plan, mask


@pytest.mark.parametrize("m", [150, 250])
def test_foe_on_long_rows(m):
    """Rows of 300 / 450 entries (m = 150: eight waves per row) and 500 / 750
    (m = 250: four waves per row), each longer than one 256-entry batch of the
    product kernel; seeded S = I + small symmetric part and H = spread
    diagonal + symmetric part, on the closed-form pattern."""
    n = 3 * m
    _print(f"case: FOE on three clusters of {m} boxes ({n} functions)")
    ctx, plan, mask = _cluster_plan(m)
    zin = torch.zeros(max(1, plan.info["in_coefs"]), dtype=torch.float64, device="cuda")
    zout = torch.zeros(max(1, plan.info["out_coefs"]), dtype=torch.float64, device="cuda")
    rows, cols = np.nonzero(mask)
    rp = np.concatenate([[0], np.cumsum(mask.sum(1))])
    for ket_out in (False, True):
        prp, pcl, _ = W.sparse_overlap(plan, zin, zout if ket_out else zin, ket_out,
                                       values=False)
        assert np.array_equal(prp.cpu().numpy(), rp) and np.array_equal(pcl.cpu().numpy(), cols)
    rng = np.random.default_rng(4100 + m)
    R1, R2 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    S = (np.eye(n) + 0.2 / np.sqrt(n) * (R1 + R1.T)) * mask
    H = (np.diag(np.linspace(-1.0, 1.0, n)) + 0.5 / np.sqrt(n) * (R2 + R2.T)) * mask
    npl, delta, nocc = 40, 0.3, 0.5 * n
    K, mu, ebs, bnd = F.foe(S, H, mask, npl, delta, nocc)
    ktol, mtol = _tolerances(bnd, delta)
    sv = torch.tensor(S[rows, cols], device="cuda")
    hv = torch.tensor(H[rows, cols], device="cuda")
    want = K[rows, cols]
    res = []
    for keep in (True, False):
        kv, gmu, gebs = W.foe(plan, sv, hv, npl, delta, nocc, keep=keep)
        got = kv.cpu().numpy()
        _print(f"  keep {keep}: K err {np.max(np.abs(got - want)):.2e} of max |K| "
               f"{np.max(np.abs(want)):.2f}, mu err {abs(gmu - mu):.2e}, "
               f"E_BS err {abs(gebs - ebs):.2e}")
        assert np.max(np.abs(got - want)) <= ktol * np.max(np.abs(want)), keep
        assert abs(gmu - mu) <= mtol and abs(gebs - ebs) <= 1e-10 * max(1.0, abs(ebs)), keep
        res.append((got, gmu, gebs))
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1:] == res[1][1:]


def test_foe_full_size_lattice():
    """The bench's FOE configuration (1,000 functions, npl = 100, delta = 1,
    n_occ = n/2, Gershgorin bounds) on a 10 x 10 x 10 lattice of 11^3 boxes
    spaced 4 points apart: boxes meet iff their lattice indices differ by at
    most 2 along every axis, so the overlap pattern (27 to 125 entries per
    row) is known in closed form and checked bit for bit.  Seeded S and H as
    in the cluster test; the oracle runs the dense masked recursion."""
    _print("case: FOE full size, 1,000 functions on a lattice, npl 100")
    L = 10
    idx = np.array([(i, j, k) for k in range(L) for j in range(L) for i in range(L)])
    lrs = [LR.box_locreg((4 * i, 4 * j, 4 * k), (11, 11, 11), (4 * i + 4, 4 * j + 4, 4 * k + 4),
                         (4 * i + 6, 4 * j + 6, 4 * k + 6)) for i, j, k in idx]
    ctx = W.Context(0.45, (48, 48, 48))
    rec, segs = to_abi(lrs)
    plan = W.Plan(ctx, rec, segs)
    n = len(lrs)
    mask = np.all(np.abs(idx[:, None, :] - idx[None, :, :]) <= 2, axis=2)
    rows, cols = np.nonzero(mask)
    rp = np.concatenate([[0], np.cumsum(mask.sum(1))])
    zin = torch.zeros(plan.info["in_coefs"], dtype=torch.float64, device="cuda")
    zout = torch.zeros(plan.info["out_coefs"], dtype=torch.float64, device="cuda")
    for ket_out in (False, True):
        prp, pcl, _ = W.sparse_overlap(plan, zin, zout if ket_out else zin, ket_out,
                                       values=False)
        assert np.array_equal(prp.cpu().numpy(), rp) and np.array_equal(pcl.cpu().numpy(), cols)
    rng = np.random.default_rng(4300)
    R1, R2 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    S = (np.eye(n) + 0.02 * (R1 + R1.T)) * mask
    H = (np.diag(np.linspace(-1.0, 1.0, n)) + 0.05 * (R2 + R2.T)) * mask
    npl, delta, nocc = 100, 1.0, 0.5 * n
    K, mu, ebs, bnd = F.foe(S, H, mask, npl, delta, nocc)
    ktol, mtol = _tolerances(bnd, delta)
    kv, gmu, gebs = W.foe(plan, torch.tensor(S[rows, cols], device="cuda"),
                          torch.tensor(H[rows, cols], device="cuda"), npl, delta, nocc)
    want = K[rows, cols]
    _print(f"  K err {np.max(np.abs(kv.cpu().numpy() - want)):.2e} of max |K| "
           f"{np.max(np.abs(want)):.2f}, mu err {abs(gmu - mu):.2e}, E_BS err {abs(gebs - ebs):.2e}")
    assert np.max(np.abs(kv.cpu().numpy() - want)) <= ktol * np.max(np.abs(want))
    assert abs(gmu - mu) <= mtol and abs(gebs - ebs) <= 1e-10 * max(1.0, abs(ebs))


def test_foe_rejects_bad_parameters(system):
    _print("case: FOE parameter checks")
    case, (srp, scl, sv), (hrp, hcl, hv) = system
    ctx = W.Context(case.g.h, case.g.grid_n)
    plan = W.Plan(ctx, case.rec, case.segs)
    s, h = torch.tensor(sv, device="cuda"), torch.tensor(hv, device="cuda")
    n = len(case.lrs)
    for args in ((0, 0.2, 3.0), (10, 0.0, 3.0), (10, 0.2, 0.0), (10, 0.2, float(n))):
        with pytest.raises(W.WvlError):
            W.foe(plan, s, h, *args)
    small = torch.empty(W.foe_scratch_bytes(plan, 10, keep=False) - 8, dtype=torch.uint8,
                        device="cuda")
    with pytest.raises(W.WvlError):
        W.foe(plan, s, h, 10, 0.2, 3.0, scratch=small)


def test_foe_spectrum_guard():
    """Tight Gershgorin bounds with the Taylor S^-1/2: S = I plus 0.4 on the
    pairs (2k, 2k + 1) of one cluster, H = -8 I plus a small symmetric part,
    on the three-cluster pattern.  H~' then has eigenvalues near -1.354; the
    guard of both sides rescales it, and the oracle without the guard is
    shown to diverge on the same input."""
    m = 10
    n = 3 * m
    _print(f"case: FOE spectrum guard, {n} functions")
    ctx, plan, mask = _cluster_plan(m)
    rng = np.random.default_rng(4200)
    S = np.eye(n)
    for k in range(0, n - 1, 2):
        if mask[k, k + 1]:
            S[k, k + 1] = S[k + 1, k] = 0.4
    R = rng.standard_normal((n, n))
    H = (-8.0 * np.eye(n) + 1e-3 * (R + R.T)) * mask
    rows, cols = np.nonzero(mask)
    # half an electron above the lower 15 states: mu sits on the upper,
    # nearly degenerate level, where Tr K'(mu) is steep and mu well defined
    npl, delta, nocc = 120, 0.5, 0.5 * n + 0.5
    K, mu, ebs, bnd = F.foe(S, H, mask, npl, delta, nocc)
    ktol, mtol = _tolerances(bnd, delta)
    assert np.max(np.abs(F.foe(S, H, mask, npl, delta, nocc, guard=False)[0])) > 1e3
    want = K[rows, cols]
    assert np.max(np.abs(want)) < 2.0
    kv, gmu, gebs = W.foe(plan, torch.tensor(S[rows, cols], device="cuda"),
                          torch.tensor(H[rows, cols], device="cuda"), npl, delta, nocc)
    err = np.max(np.abs(kv.cpu().numpy() - want))
    _print(f"  K err {err:.2e} (max |K| {np.max(np.abs(want)):.2f}), mu err {abs(gmu - mu):.2e}")
    assert err <= ktol * np.max(np.abs(want))
    assert abs(gmu - mu) <= mtol and abs(gebs - ebs) <= 1e-10 * max(1.0, abs(ebs))
