"""Fermi operator expansion (paper Sec. IV.B, App. B) through the C ABI
against the oracle, on S and H computed by the oracle (the same values feed
both sides).  Tolerance: both sides run the same steps in double with sums
in different orders and independently computed coefficients and bisections,
so K agrees to 1e-9 of its largest entry, mu to 1e-9 and E_BS to 1e-9
relative."""
import numpy as np
import pytest

from oracle import foe as F
from oracle import sparse as SP
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
    K, mu, ebs, _ = F.foe(S, H, mask, npl, delta, nocc, emin, emax)
    kv, gmu, gebs = W.foe(plan, torch.tensor(sv, device="cuda"), torch.tensor(hv, device="cuda"),
                          npl, delta, nocc, emin or 0.0, emax or 0.0)
    got = kv.cpu().numpy()
    want = np.array([K[a, scl[q]] for a in range(n) for q in range(srp[a], srp[a + 1])])
    assert np.max(np.abs(got - want)) <= 1e-9 * np.max(np.abs(want))
    assert abs(gmu - mu) <= 1e-9
    assert abs(gebs - ebs) <= 1e-9 * max(1.0, abs(ebs))
    # bitwise reproducible
    kv2, mu2, ebs2 = W.foe(plan, torch.tensor(sv, device="cuda"), torch.tensor(hv, device="cuda"),
                           npl, delta, nocc, emin or 0.0, emax or 0.0)
    assert np.array_equal(kv2.cpu().numpy(), got) and mu2 == gmu and ebs2 == gebs


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
