"""The allocation-free apply (wvl_apply_local_ham_static, workspace in a
static device array of the library) through the C ABI, against
wvl_apply_local_ham on the same plans and inputs: two calls in a row, the
second with a smaller input, each giving the same bits as the entry point
with a caller workspace (the same kernels in the same layout), and the
smaller one also against the oracle to the parity tolerances (FP64 1e-12,
FP32 1e-5 relative; FP32 energies 1e-6 Ha).  A plan that needs more than the
static workspace is rejected before anything runs."""
import numpy as np
import pytest

import inputs
from oracle import locreg as LR
from tests.abi_helpers import rel_err
from tests.test_gpu_parity import Case, _print, _sphere_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1401_7441_amd as W


def _batch_case(nsf):
    g = inputs.geometry("batch1k", nsf=nsf, seed_offset=11)
    lrs = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
    return Case(g, lrs)


def _both(case, dtype, max_ws):
    ctx = W.Context(case.g.h, case.g.grid_n)
    plan = W.Plan(ctx, case.rec, case.segs, max_workspace=max_ws)
    psi = torch.tensor(case.psi, dtype=dtype, device="cuda")
    pot = torch.tensor(case.pot, dtype=dtype, device="cuda")
    n = len(case.lrs)
    outs = []
    for static in (False, True):
        out = torch.full((plan.info["out_coefs"],), float("nan"), dtype=dtype, device="cuda")
        ek = torch.zeros(n, dtype=torch.float64, device="cuda")
        ep = torch.zeros_like(ek)
        if static:
            W.apply_local_ham_static(plan, psi, pot, out, ek, ep)
        else:
            W.apply_local_ham(plan, psi, pot, out, ek, ep)
        torch.cuda.synchronize()
        outs.append((out.cpu().numpy(), ek.cpu().numpy(), ep.cpu().numpy()))
    return plan, outs


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_static_apply_two_calls_second_smaller(dtype):
    big = _batch_case(12)                  # batch1k-size boxes, chunked
    small = _sphere_case(nsf=3, seed_shift=21)
    ws_bound = 96 << 20
    for name, case, bound in (("12 batch1k functions", big, ws_bound),
                              ("3 small functions", small, 0)):
        _print(f"case: static-workspace apply, {name}, {dtype}")
        plan, (ref, got) = _both(case, dtype, bound)
        code = W.F64 if dtype == torch.float64 else W.F32
        assert plan.workspace_bytes(code) <= W.STATIC_WORKSPACE_BYTES
        for r, g in zip(ref, got):
            assert np.array_equal(r, g)
        out, ek, ep = got
        tol = 1e-12 if dtype == torch.float64 else 1e-5
        for k in range(len(case.lrs)):
            oh, oek, oep = case.oracle(k)
            assert rel_err(out[case.out_slice(k)], oh) < tol, k
            etol = 1e-12 * max(1.0, abs(oek)) if dtype == torch.float64 else 1e-6
            assert abs(ek[k] - oek) <= etol and abs(ep[k] - oep) <= max(etol, 1e-12), k
        if name.startswith("12"):
            assert plan.info["chunks"] > 1


def test_static_apply_rejects_large_plans():
    _print("case: static-workspace apply rejects a plan larger than the static workspace")
    case = _batch_case(12)
    ctx = W.Context(case.g.h, case.g.grid_n)
    plan = W.Plan(ctx, case.rec, case.segs)             # one chunk: about 30 MB per function
    assert plan.workspace_bytes(W.F64) > W.STATIC_WORKSPACE_BYTES
    psi = torch.tensor(case.psi, dtype=torch.float64, device="cuda")
    pot = torch.tensor(case.pot, dtype=torch.float64, device="cuda")
    out = torch.zeros(plan.info["out_coefs"], dtype=torch.float64, device="cuda")
    with pytest.raises(W.WvlError) as e:
        W.apply_local_ham_static(plan, psi, pot, out)
    assert e.value.status == W.WVL_EINVAL and "static" in str(e.value)
