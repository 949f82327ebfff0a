"""The 1,000-function batch at full size, in the launch configuration the
benchmark times (its own set-up, the autotuned layout, the captured step
replayed as a graph), against the oracle on sampled outputs the oracle
computes one by one:

* the library's segments equal the oracle's, for every function (bit-exact);
* H|phi>, e_kin and e_pot of sampled functions (FP64 1e-12, FP32 1e-5
  relative; FP32 energies within 1e-6 Ha per normalized function);
* sampled rows of the S and H patterns (bit-exact) and their values
  (|dS_ab| <= tol |phi_a| |phi_b|, |dH_ab| <= tol |phi_a| |H phi_b|).
"""
import numpy as np
import pytest

import inputs
from oracle import hamiltonian as Hm
from oracle import locreg as LR
from oracle import sparse as SP
from tests.abi_helpers import rel_err, to_abi
from tests.test_gpu_parity import _print

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1401_7441_amd as W

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def oracle_side():
    g = inputs.geometry("batch1k")
    lrs = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
    return g, lrs, inputs.potential(g).numpy()


def _coef(g, lrs, k):
    l = lrs[k]
    return inputs.coefficients(g, k, LR.points_from_segments(l.cseg),
                               LR.points_from_segments(l.fseg))


def _row(lrs, a, ket_out):
    """The oracle's pattern row a (exact set test after a box filter)."""
    bra_box = SP._bbox(lrs[a].cseg)
    cols = []
    for b, lb in enumerate(lrs):
        kseg = lb.ocseg if ket_out else lb.cseg
        if SP._boxes_meet(bra_box, SP._bbox(kseg)) and SP.pair_intersects(lrs[a].cseg, kseg):
            cols.append(b)
    return np.array(cols)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch1k_full_size_sampled(oracle_side, dtype):
    import bench
    _print(f"case: batch1k full size, {dtype}, benchmark launch configuration")
    g, lrs, pot = oracle_side
    S = bench.setup("batch1k", dtype)
    plan, n = S["plan"], len(lrs)
    rec, segs = to_abi(lrs)
    assert np.array_equal(S["segs"], segs)
    for f in ("seg_c", "nseg_c", "seg_f", "nseg_f", "oseg_c", "noseg_c", "oseg_f", "noseg_f",
              "coef_off", "ocoef_off", "lo", "dims"):
        assert np.array_equal(S["lr"][f], rec[f]), f
    W.autotune(plan, S["psi"], S["pot"], S["hpsi"], S["ws"], reps=1)
    graph = W.Graph(plan, S["psi"], S["pot"], S["hpsi"], S["ek"], S["ep"], workspace=S["ws"],
                    s_val=S["s_out"][2], h_val=S["h_out"][2])
    graph.launch()
    torch.cuda.synchronize()
    out = S["hpsi"].cpu().numpy().astype(np.float64)
    ek, ep = S["ek"].cpu().numpy(), S["ep"].cpu().numpy()
    sval, hval = S["s_out"][2].cpu().numpy(), S["h_out"][2].cpu().numpy()
    srp, scl, _ = W.sparse_overlap(plan, S["psi"], S["psi"], False, values=False)
    hrp, hcl, _ = W.sparse_overlap(plan, S["psi"], S["hpsi"], True, values=False)
    srp, scl, hrp, hcl = (t.cpu().numpy() for t in (srp, scl, hrp, hcl))
    graph.close()
    vol = [int(np.prod(l.dims)) for l in lrs]
    sample = sorted({0, n // 2, n - 1, int(np.argmax(vol)), int(np.argmin(vol))})
    tol = TOL[dtype]
    coefs, ohs = {}, {}
    for k in sample:
        coefs[k] = _coef(g, lrs, k)
        oh, oek, oep = Hm.apply_local_ham(lrs[k], coefs[k], pot, g.h)
        ohs[k] = oh
        r = rec[k]
        got = out[int(r["ocoef_off"]):int(r["ocoef_off"]) + int(r["on_c"]) + 7 * int(r["on_f"])]
        assert rel_err(got, oh) < tol, (k, rel_err(got, oh))
        etol = 1e-6 if dtype == "f32" else 1e-12 * max(1.0, abs(oek))
        assert abs(ek[k] - oek) <= etol, (k, ek[k], oek)
        assert abs(ep[k] - oep) <= (1e-6 if dtype == "f32" else 1e-12 * max(1.0, abs(oep))), k
    # S rows of two sampled functions, H columns of two sampled kets
    for a in sample[:2]:
        cols = _row(lrs, a, False)
        assert np.array_equal(scl[srp[a]:srp[a + 1]], cols), a
        na = np.linalg.norm(coefs[a])
        for q in range(srp[a], srp[a + 1]):
            b = int(scl[q])
            cb = coefs[b] if b in coefs else _coef(g, lrs, b)
            want = SP.pair_value((lrs[a].cseg, lrs[a].fseg), coefs[a],
                                 (lrs[b].cseg, lrs[b].fseg), cb)
            assert abs(sval[q] - want) <= tol * na * np.linalg.norm(cb), (a, b)
    for b in sample[-2:]:
        nh = np.linalg.norm(ohs[b])
        rows = [a for a in range(n) if b in hcl[hrp[a]:hrp[a + 1]]]
        assert rows, b
        for i, a in enumerate(rows[:40]):
            if i < 4:
                assert np.array_equal(hcl[hrp[a]:hrp[a + 1]], _row(lrs, a, True)), a
            q = hrp[a] + int(np.searchsorted(hcl[hrp[a]:hrp[a + 1]], b))
            ca = coefs[a] if a in coefs else _coef(g, lrs, a)
            want = SP.pair_value((lrs[a].cseg, lrs[a].fseg), ca,
                                 (lrs[b].ocseg, lrs[b].ofseg), ohs[b])
            assert abs(hval[q] - want) <= tol * np.linalg.norm(ca) * nh, (a, b)
