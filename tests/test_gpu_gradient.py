"""wvl_gradient (Eq. (gradient), Sec. IV.A) through the C ABI against the
oracle.  Inputs on both sides: seeded coefficients psi, seeded vectors on
the output patterns standing in for H|phi> (the operation is defined for
any such vectors), S and H formed by the oracle from them (small case) or
seeded values on the patterns (the 1,000-function case), a symmetric kernel
K on the overlap pattern.  Tolerances: the coefficient matrices are sums of
products in double in another order (1e-12 relative to the largest entry);
the gradient FP64 1e-12, FP32 1e-5 relative per function."""
import numpy as np
import pytest

from oracle import gradient as G
from oracle import locreg as LR
from oracle import sparse as SP
from tests.abi_helpers import rel_err, to_abi
from tests.test_gpu_parity import _print, _sphere_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1401_7441_amd as W


def _dense(n, rp, cl, vv):
    A = np.zeros((n, n))
    for a in range(n):
        A[a, cl[rp[a]:rp[a + 1]]] = vv[rp[a]:rp[a + 1]]
    return A


def _run(case, psi, hpsi, sv, hv, kv, dtype):
    ctx = W.Context(case.g.h, case.g.grid_n)
    plan = W.Plan(ctx, case.rec, case.segs)
    p = torch.tensor(np.concatenate(psi), dtype=dtype, device="cuda")
    hp = torch.tensor(np.concatenate(hpsi), dtype=dtype, device="cuda")
    g = W.gradient(plan, torch.tensor(sv, device="cuda"), torch.tensor(hv, device="cuda"),
                   torch.tensor(kv, device="cuda"), p, hp)
    g2 = W.gradient(plan, torch.tensor(sv, device="cuda"), torch.tensor(hv, device="cuda"),
                    torch.tensor(kv, device="cuda"), p, hp)
    torch.cuda.synchronize()
    out = g.cpu().numpy().astype(np.float64)
    assert np.array_equal(out, g2.cpu().numpy().astype(np.float64))   # bitwise repeatable
    return plan, out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gradient_against_oracle(dtype):
    _print(f"case: gradient, 8 functions, {dtype}")
    case = _sphere_case(nsf=8, seed_shift=31)
    n = len(case.lrs)
    rng = np.random.default_rng(310)
    psi = case.coefs
    hpsi = [rng.standard_normal(l.on_c + 7 * l.on_f) / np.sqrt(l.on_c + 7 * l.on_f)
            for l in case.lrs]
    srp, scl, sv = SP.matrix(case.lrs, psi, psi, False)
    hrp, hcl, hv = SP.matrix(case.lrs, psi, hpsi, True)
    mask = _dense(n, srp, scl, np.ones(len(scl))) > 0
    Kd = rng.standard_normal((n, n)) * 0.3
    Kd = (Kd + Kd.T) * mask
    kv = Kd[mask]
    A, M = G.coefficient_matrices(_dense(n, srp, scl, sv), _dense(n, hrp, hcl, hv), Kd, mask)
    want = G.gradient(case.lrs, psi, hpsi, A, M, mask)
    dt = torch.float64 if dtype == "f64" else torch.float32
    _, got = _run(case, psi, hpsi, sv, hv, kv, dt)
    tol = 1e-12 if dtype == "f64" else 1e-5
    off = np.cumsum([0] + [l.n_c + 7 * l.n_f for l in case.lrs])
    errs = [rel_err(got[off[a]:off[a + 1]], want[a]) for a in range(n)]
    _print(f"  worst relative error {max(errs):.2e}")
    assert max(errs) < tol, errs


def test_gradient_full_size_sampled():
    """1,000 functions on a 10 x 10 x 10 lattice of 11^3 boxes spaced 4
    points apart (fine sub-box 3^3, output = input pattern): boxes meet iff
    their lattice indices differ by at most 2 on every axis, so the overlap
    pattern is known in closed form (checked bit for bit against the
    library's).  FP64; the oracle forms the coefficient matrices densely and
    the gradient of sampled rows."""
    _print("case: gradient, 1,000 functions on a lattice, sampled rows")
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
    rng = np.random.default_rng(320)
    psi = [rng.standard_normal(l.n_c + 7 * l.n_f) * 0.03 for l in lrs]
    hpsi = [rng.standard_normal(l.on_c + 7 * l.on_f) * 0.03 for l in lrs]
    pt = torch.tensor(np.concatenate(psi), device="cuda")
    ht = torch.tensor(np.concatenate(hpsi), device="cuda")
    for ket_out in (False, True):
        prp, pcl, _ = W.sparse_overlap(plan, pt, ht if ket_out else pt, ket_out, values=False)
        assert np.array_equal(pcl.cpu().numpy(), cols)
    R = rng.standard_normal((n, n)) * 0.02
    Sd = (np.eye(n) + R + R.T) * mask
    Hd = rng.standard_normal((n, n)) * mask
    R = rng.standard_normal((n, n)) * 0.1
    Kd = (R + R.T) * mask
    gt = W.gradient(plan, torch.tensor(Sd[rows, cols], device="cuda"),
                    torch.tensor(Hd[rows, cols], device="cuda"),
                    torch.tensor(Kd[rows, cols], device="cuda"), pt, ht)
    torch.cuda.synchronize()
    got = gt.cpu().numpy()
    A, M = G.coefficient_matrices(Sd, Hd, Kd, mask)
    sample = sorted(set(int(k) for k in rng.choice(n, 6, replace=False)) | {0, 555, n - 1})
    want = G.gradient(lrs, psi, hpsi, A, M, mask, rows=sample)
    off = np.cumsum([0] + [l.n_c + 7 * l.n_f for l in lrs])
    worst = 0.0
    for a, w in zip(sample, want):
        e = rel_err(got[off[a]:off[a + 1]], w)
        worst = max(worst, e)
        assert e < 1e-12, (a, e)
    _print(f"  {len(sample)} rows, worst relative error {worst:.2e}")
