"""Parity at the workloads the benchmark runs, in its launch configuration
(its set-up, the autotuned layout, the captured step replayed as a graph),
against the oracle on sampled outputs the oracle computes one by one:

* gpu16k (16,000 functions in a 110 bohr cube, FP32 convolutions, FP64
  S/H): H|phi>, e_kin and e_pot of a seeded sample of 32 functions plus the
  smallest and largest box; their S and H pattern rows (bit-exact, from the
  oracle's own coarse sets); S values and H values (as kets) on sampled
  entries of those rows;
* sweep2k (2,000 cubic boxes of 16^3 to 48^3 coarse points), FP32 and FP64:
  the same on a sample that holds a 16^3 and a 48^3 box;
* smooth, envelope-only, normalized functions of batch1k size in FP32: e_kin
  and e_pot within 1e-6 Ha of the oracle (the case the difference form of
  the FP32 kinetic filter exists for).

Tolerances as in tests/test_gpu_parity.py: H|phi> per function 1e-12 (FP64)
or 1e-5 (FP32) relative; energies 1e-12 relative (FP64) or 1e-6 Ha per
normalized function (FP32); |dS_ab| <= tol |phi_a| |phi_b|,
|dH_ab| <= tol |phi_a| |H phi_b|.
"""
import numpy as np
import pytest

import inputs
from oracle import hamiltonian as Hm
from oracle import locreg as LR
from oracle import sparse as SP
from tests.abi_helpers import rel_err
from tests.test_gpu_parity import Case, _print

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1401_7441_amd as W

TOL = {"f32": 1e-5, "f64": 1e-12}


def _meets(A, B):
    """Do two coarse sets (mask[z, y, x], origin) share a grid point?"""
    (ma, la), (mb, lb) = A, B
    lo = [max(la[a], lb[a]) for a in range(3)]
    hi = [min(la[a] + ma.shape[2 - a], lb[a] + mb.shape[2 - a]) for a in range(3)]
    if any(hi[a] <= lo[a] for a in range(3)):
        return False
    sa = ma[lo[2] - la[2]:hi[2] - la[2], lo[1] - la[1]:hi[1] - la[1], lo[0] - la[0]:hi[0] - la[0]]
    sb = mb[lo[2] - lb[2]:hi[2] - lb[2], lo[1] - lb[1]:hi[1] - lb[1], lo[0] - lb[0]:hi[0] - lb[0]]
    return bool(np.any(sa & sb))


class Oracle:
    """The oracle's side of a workload: sphere sets, locregs and coefficients
    built on demand for the functions a test samples."""

    def __init__(self, workload):
        g = inputs.geometry(workload)
        self.g = g
        self.spheres = LR.SphereSet(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
        self.pot = inputs.potential(g).numpy()
        self._lr, self._c, self._set = {}, {}, {}

    def lr(self, k):
        if k not in self._lr:
            self._lr[k] = self.spheres.locreg(k)
        return self._lr[k]

    def coef(self, k):
        if k not in self._c:
            l = self.lr(k)
            self._c[k] = inputs.coefficients(self.g, k, LR.points_from_segments(l.cseg),
                                             LR.points_from_segments(l.fseg))
        return self._c[k]

    def cset(self, k, out):
        if (k, out) not in self._set:
            self._set[(k, out)] = self.spheres.coarse_set(k, out)
        return self._set[(k, out)]

    def row(self, a, ket_out):
        """Pattern row a: the kets whose (input or output) coarse set meets
        a's input coarse set, found by intersecting the oracle's sets of the
        functions whose spheres can reach a's."""
        g = self.g
        reach = g.radii[a] + g.radii + (g.ext * g.h if ket_out else 0.0) + 2.0 * g.h
        d = np.linalg.norm(g.centers - g.centers[a], axis=1)
        cand = np.nonzero(d <= reach)[0]
        return np.array([b for b in cand if _meets(self.cset(a, False), self.cset(b, ket_out))],
                        np.int64)

    def col(self, b):
        """Column b of the H pattern: the bras whose input coarse set meets
        b's output coarse set."""
        g = self.g
        reach = g.radii[b] + g.radii + g.ext * g.h + 2.0 * g.h
        d = np.linalg.norm(g.centers - g.centers[b], axis=1)
        cand = np.nonzero(d <= reach)[0]
        return np.array([a for a in cand if _meets(self.cset(a, False), self.cset(b, True))],
                        np.int64)


def _graph_run(workload, dtype):
    """The benchmark's set-up, autotuner and one graph replay of the step."""
    import bench
    torch.cuda.empty_cache()
    S = bench.setup(workload, dtype)
    W.autotune(S["plan"], S["psi"], S["pot"], S["hpsi"], S["ws"], reps=1)
    graph = W.Graph(S["plan"], S["psi"], S["pot"], S["hpsi"], S["ek"], S["ep"],
                    workspace=S["ws"], s_val=S["s_out"][2], h_val=S["h_out"][2])
    graph.launch()
    torch.cuda.synchronize()
    plan = S["plan"]
    srp, scl, _ = W.sparse_overlap(plan, S["psi"], S["psi"], False, values=False)
    hrp, hcl, _ = W.sparse_overlap(plan, S["psi"], S["hpsi"], True, values=False)
    res = {"lr": S["lr"], "ek": S["ek"].cpu().numpy(), "ep": S["ep"].cpu().numpy(),
           "sval": S["s_out"][2].cpu().numpy(), "hval": S["h_out"][2].cpu().numpy(),
           "srp": srp.cpu().numpy(), "scl": scl.cpu().numpy(), "hrp": hrp.cpu().numpy(),
           "hcl": hcl.cpu().numpy(), "hpsi": S["hpsi"], "psi": S["psi"]}
    graph.close()
    return S, res


def _check_sampled(O, R, sample, dtype, n_entries=4, seed=0):
    tol = TOL[dtype]
    rng = np.random.default_rng(seed)
    lr = R["lr"]
    srp, scl, hrp, hcl = R["srp"], R["scl"], R["hrp"], R["hcl"]
    worst = {"hpsi": 0.0, "ek": 0.0, "ep": 0.0, "s": 0.0, "h": 0.0}
    for k in sample:
        r = lr[k]
        o, n = int(r["ocoef_off"]), int(r["on_c"]) + 7 * int(r["on_f"])
        got = R["hpsi"][o:o + n].cpu().numpy().astype(np.float64)
        oh, oek, oep = Hm.apply_local_ham(O.lr(k), O.coef(k), O.pot, O.g.h)
        e = rel_err(got, oh)
        worst["hpsi"] = max(worst["hpsi"], e)
        assert e < tol, (k, e)
        if dtype == "f32":
            ek_tol, ep_tol = 1e-6, 1e-6
        else:
            ek_tol, ep_tol = 1e-12 * max(1.0, abs(oek)), 1e-12 * max(1.0, abs(oep))
        worst["ek"] = max(worst["ek"], abs(R["ek"][k] - oek))
        worst["ep"] = max(worst["ep"], abs(R["ep"][k] - oep))
        assert abs(R["ek"][k] - oek) <= ek_tol, (k, R["ek"][k], oek)
        assert abs(R["ep"][k] - oep) <= ep_tol, (k, R["ep"][k], oep)
        # pattern rows of k, bit-exact
        assert np.array_equal(scl[srp[k]:srp[k + 1]], O.row(k, False)), k
        assert np.array_equal(hcl[hrp[k]:hrp[k + 1]], O.row(k, True)), k
        # S_kb on the diagonal and a few sampled entries of row k
        ca, la = O.coef(k), O.lr(k)
        qs = np.unique(np.concatenate([[srp[k] + int(np.searchsorted(scl[srp[k]:srp[k + 1]], k))],
                                       rng.integers(srp[k], srp[k + 1], n_entries)]))
        for q in qs:
            b = int(scl[q])
            want = SP.pair_value((la.cseg, la.fseg), ca, (O.lr(b).cseg, O.lr(b).fseg), O.coef(b))
            bound = tol * np.linalg.norm(ca) * np.linalg.norm(O.coef(b))
            worst["s"] = max(worst["s"], abs(R["sval"][q] - want) / bound * tol)
            assert abs(R["sval"][q] - want) <= bound, (k, b)
        # column k of H (bit-exact) and H_ak with k as the ket, for a few rows
        cand = np.searchsorted(hrp, np.nonzero(hcl == k)[0], side="right") - 1
        assert np.array_equal(cand, O.col(k)), k
        assert k in cand
        for a in np.unique(np.concatenate([[k], rng.choice(cand, min(n_entries, len(cand)),
                                                          replace=False)])):
            a = int(a)
            q = hrp[a] + int(np.searchsorted(hcl[hrp[a]:hrp[a + 1]], k))
            assert hcl[q] == k
            want = SP.pair_value((O.lr(a).cseg, O.lr(a).fseg), O.coef(a),
                                 (O.lr(k).ocseg, O.lr(k).ofseg), oh)
            bound = tol * np.linalg.norm(O.coef(a)) * np.linalg.norm(oh)
            worst["h"] = max(worst["h"], abs(R["hval"][q] - want) / bound * tol)
            assert abs(R["hval"][q] - want) <= bound, (a, k)
    return worst


def _sample(lr, n, seed):
    vol = np.prod(np.asarray(lr["dims"], np.int64), axis=1)
    rng = np.random.default_rng(seed)
    pick = set(int(k) for k in rng.choice(len(lr), n, replace=False))
    pick |= {int(np.argmin(vol)), int(np.argmax(vol))}
    return sorted(pick), vol


def test_gpu16k_sampled():
    _print("case: gpu16k (16,000 functions), f32, benchmark launch configuration")
    O = Oracle("gpu16k")
    S, R = _graph_run("gpu16k", "f32")
    sample, _ = _sample(R["lr"], 32, 16000)
    worst = _check_sampled(O, R, sample, "f32")
    _print(f"  {len(sample)} functions, worst errors {worst}")
    del S, R


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_sweep2k_sampled(dtype):
    _print(f"case: sweep2k (boxes 16^3 to 48^3), {dtype}, benchmark launch configuration")
    O = Oracle("sweep2k")
    S, R = _graph_run("sweep2k", dtype)
    sample, vol = _sample(R["lr"], 8, 2000)
    dims = np.asarray(R["lr"]["dims"])
    # the sample holds the smallest and the largest box of the workload
    # (spheres of box edge 16 and 48 have 15-16 and 47 points along an axis)
    assert dims[sample].max() >= 47 and dims[sample].min() <= 16, dims[sample]
    _print(f"  boxes {sorted(set(int(d) for d in dims[sample].max(1)))}")
    worst = _check_sampled(O, R, sample, dtype, n_entries=3)
    _print(f"  {len(sample)} functions, worst errors {worst}")
    del S, R


def test_smooth_functions_fp32_energies():
    """Envelope-only coefficients, normalized: the kinetic filter's
    cancellation is largest here; FP32 energies stay within 1e-6 Ha."""
    _print("case: smooth normalized functions, FP32 energies")
    g = inputs.geometry("batch1k", nsf=8, seed_offset=3)
    lrs = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
    case = Case(g, lrs, smooth=True)
    _, _, out, ek, ep = case.run(torch.float32)
    worst = [0.0, 0.0, 0.0]
    for k in range(len(lrs)):
        ref, rk, rp = case.oracle(k)
        worst = [max(worst[0], rel_err(out[case.out_slice(k)], ref)),
                 max(worst[1], abs(ek[k] - rk)), max(worst[2], abs(ep[k] - rp))]
        assert rel_err(out[case.out_slice(k)], ref) < 1e-5, k
        assert abs(ek[k] - rk) <= 1e-6, (k, ek[k], rk)
        assert abs(ep[k] - rp) <= 1e-6, (k, ep[k], rp)
    _print(f"  worst: H|phi> {worst[0]:.2e}, e_kin {worst[1]:.2e} Ha, e_pot {worst[2]:.2e} Ha")
