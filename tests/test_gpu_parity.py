"""GPU parity: the HIP library against the FP64 oracle, through the C ABI.

Tolerances (stated by the target and derived in the design notes):
  FP64 path: per-function relative L2 error of H|phi> <= 1e-12; energies and
             matrix elements relative 1e-12.
  FP32 path: per-function relative L2 error <= 1e-5; energies within 1e-6 Ha
             per normalized function; matrix elements |dS_ab| <= 1e-5
             sqrt(S_aa S_bb), |dH_ab| <= 1e-5 |phi_a| |H phi_b|.
  Index work (segments, patterns, uncompress/compress) is bit-exact."""
import math

import numpy as np
import pytest

import inputs
from oracle import hamiltonian as Hm
from oracle import locreg as LR
from oracle import sparse as SP
from tests.abi_helpers import from_abi, rel_err, to_abi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1401_7441_amd as W


def _print(*a):
    print(*a, flush=True)


class Case:
    """A batch of support functions: oracle locregs, coefficients, potential."""

    def __init__(self, g, lrs, smooth=False, normalize=True):
        self.g = g
        self.lrs = lrs
        self.rec, self.segs = to_abi(lrs)
        self.coefs = []
        for k, l in enumerate(lrs):
            pc = LR.points_from_segments(l.cseg)
            pf = LR.points_from_segments(l.fseg)
            self.coefs.append(inputs.coefficients(g, k, pc, pf, smooth=smooth,
                                                  normalize=normalize))
        self.psi = np.concatenate(self.coefs) if self.coefs else np.zeros(0)
        self.pot = inputs.potential(g).numpy()

    def oracle(self, k, **kw):
        key = (k, tuple(sorted(kw.items())))
        if not hasattr(self, "_memo"):
            self._memo = {}
        if key not in self._memo:
            self._memo[key] = Hm.apply_local_ham(self.lrs[k], self.coefs[k], self.pot, self.g.h,
                                                 **kw)
        return self._memo[key]

    def run(self, dtype, terms=None, max_workspace=0, plan=None):
        ctx = W.Context(self.g.h, self.g.grid_n)
        plan = plan or W.Plan(ctx, self.rec, self.segs, max_workspace=max_workspace)
        psi = torch.tensor(self.psi, dtype=dtype, device="cuda")
        pot = torch.tensor(self.pot, dtype=dtype, device="cuda")
        out = torch.zeros(plan.info["out_coefs"], dtype=dtype, device="cuda")
        ek = torch.zeros(len(self.lrs), dtype=torch.float64, device="cuda")
        ep = torch.zeros_like(ek)
        W.apply_local_ham(plan, psi, pot, out, ek, ep, terms=terms or (W.KIN | W.POT))
        torch.cuda.synchronize()
        return plan, psi, out.cpu().numpy(), ek.cpu().numpy(), ep.cpu().numpy()

    def out_slice(self, k):
        r = self.rec[k]
        n = int(r["on_c"]) + 7 * int(r["on_f"])
        return slice(int(r["ocoef_off"]), int(r["ocoef_off"]) + n)


def _single_case():
    g = inputs.geometry("single")
    lo, dims, flo, fhi = inputs.single_box()
    return Case(g, [LR.box_locreg(lo, dims, flo, fhi)], normalize=True)


def _sphere_case(nsf=6, rlo=2.4, rhi=3.4, ext=8, seed_shift=0, fine=1.6):
    g = inputs.geometry("batch1k", nsf=nsf, seed_offset=seed_shift)
    rng = np.random.default_rng(99 + seed_shift)
    # pull the centres together so that the functions overlap
    g.centers[:] = g.centers.mean(0) + rng.uniform(-4.0, 4.0, (nsf, 3))
    g.radii[:] = rng.uniform(rlo, rhi, nsf)
    g.fine_radii[:] = fine
    g.envelope_sigma[:] = g.radii / 2
    lrs = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, ext)
    return Case(g, lrs)


@pytest.fixture(scope="module")
def single():
    return _single_case()


@pytest.fixture(scope="module")
def spheres():
    return _sphere_case()


def test_single_function_fp64(single):
    _print("case: single function, FP64")
    _, _, out, ek, ep = single.run(torch.float64)
    ref, rk, rp = single.oracle(0)
    assert rel_err(out, ref) < 1e-12
    assert abs(ek[0] - rk) < 1e-12 * abs(rk)
    assert abs(ep[0] - rp) < 1e-12 * abs(rk)
    psi = single.coefs[0]
    assert abs(psi @ out - (rk + rp)) < 1e-12 * abs(rk)


def test_single_function_fp32(single):
    _print("case: single function, FP32")
    _, _, out, ek, ep = single.run(torch.float32)
    ref, rk, rp = single.oracle(0)
    assert rel_err(out, ref) < 1e-5
    assert abs(ek[0] - rk) < 1e-6
    assert abs(ep[0] - rp) < 1e-6


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_sphere_batch_every_function(spheres, dtype, tol):
    _print(f"case: 6 overlapping spheres, ext 8, {dtype}")
    dt = torch.float64 if dtype == "f64" else torch.float32
    _, _, out, ek, ep = spheres.run(dt)
    for k in range(len(spheres.lrs)):
        ref, rk, rp = spheres.oracle(k)
        assert rel_err(out[spheres.out_slice(k)], ref) < tol, k
        etol = 1e-12 * abs(rk) if dtype == "f64" else 1e-6
        assert abs(ek[k] - rk) < etol and abs(ep[k] - rp) < etol, k


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_kinetic_z_on_matrix_cores(spheres, dtype, tol):
    """The schedule with the z part of the kinetic term as banded-Toeplitz
    products on the FP64 matrix cores (k_kin_zmfma), 1 and 3 bins: H|phi>,
    e_kin, e_pot and the kinetic term alone against the oracle."""
    _print(f"case: z kinetic on the matrix cores, {dtype}")
    dt = torch.float64 if dtype == "f64" else torch.float32
    for nbins in (1, 3):
        ctx = W.Context(spheres.g.h, spheres.g.grid_n)
        plan = W.Plan(ctx, spheres.rec, spheres.segs)
        W.set_schedule(plan, nbins, 1)
        _, _, out, ek, ep = spheres.run(dt, plan=plan)
        _, _, outk, _, _ = spheres.run(dt, terms=W.KIN, plan=plan)
        worst = 0.0
        for k in range(len(spheres.lrs)):
            ref, rk, rp = spheres.oracle(k)
            refk, _, _ = spheres.oracle(k, potential=False)
            worst = max(worst, rel_err(out[spheres.out_slice(k)], ref))
            assert rel_err(out[spheres.out_slice(k)], ref) < tol, k
            assert rel_err(outk[spheres.out_slice(k)], refk) < tol, k
            etol = 1e-12 * abs(rk) if dtype == "f64" else 1e-6
            assert abs(ek[k] - rk) < etol and abs(ep[k] - rp) < etol, k
        _print(f"  {nbins} bins: worst relative error {worst:.2e}")


def test_kinetic_and_potential_terms_separately(spheres):
    _print("case: separate terms FP64")
    _, _, outk, ek, _ = spheres.run(torch.float64, terms=W.KIN)
    _, _, outp, _, ep = spheres.run(torch.float64, terms=W.POT)
    for k in range(len(spheres.lrs)):
        refk, rk, _ = spheres.oracle(k, potential=False)
        refp, _, rp = spheres.oracle(k, kinetic=False)
        assert rel_err(outk[spheres.out_slice(k)], refk) < 1e-12
        assert rel_err(outp[spheres.out_slice(k)], refp) < 1e-12


def test_wvl_kinetic_accumulates(spheres):
    _print("case: wvl_kinetic accumulate")
    ctx = W.Context(spheres.g.h, spheres.g.grid_n)
    plan = W.Plan(ctx, spheres.rec, spheres.segs)
    psi = torch.tensor(spheres.psi, dtype=torch.float64, device="cuda")
    base = torch.arange(plan.info["out_coefs"], dtype=torch.float64, device="cuda") * 1e-3
    out = base.clone()
    W.kinetic(plan, psi, out)
    torch.cuda.synchronize()
    got = (out - base).cpu().numpy()
    for k in range(len(spheres.lrs)):
        refk, _, _ = spheres.oracle(k, potential=False)
        assert rel_err(got[spheres.out_slice(k)], refk) < 1e-12


def test_uncompress_compress_bit_exact(spheres):
    _print("case: uncompress / compress")
    ctx = W.Context(spheres.g.h, spheres.g.grid_n)
    plan = W.Plan(ctx, spheres.rec, spheres.segs)
    psi = torch.tensor(spheres.psi, dtype=torch.float64, device="cuda")
    box = torch.full((plan.info["in_box"],), float("nan"), dtype=torch.float64, device="cuda")
    W.uncompress(plan, psi, box)
    torch.cuda.synchronize()
    b = box.cpu().numpy()
    off = 0
    obox_parts = []
    for k, l in enumerate(spheres.lrs):
        ref = Hm.uncompress(l, spheres.coefs[k])
        assert np.array_equal(b[off:off + ref.size], ref.ravel()), k
        off += ref.size
        e = l.ext
        ob = np.random.default_rng(k).standard_normal(
            (8, l.dims[2] + 2 * e, l.dims[1] + 2 * e, l.dims[0] + 2 * e))
        obox_parts.append(ob)
    obox = torch.tensor(np.concatenate([o.ravel() for o in obox_parts]), device="cuda")
    out = torch.full((plan.info["out_coefs"],), float("nan"), dtype=torch.float64, device="cuda")
    W.compress(plan, obox, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for k, l in enumerate(spheres.lrs):
        assert np.array_equal(o[spheres.out_slice(k)], Hm.compress_out(l, obox_parts[k]))


def test_edge_boxes_fp64():
    """1x1x1 and anisotropic boxes, empty fine set, fine set = whole box,
    ext 0 and ext 16, a box in the grid corner (output pattern clipped)."""
    _print("case: edge boxes")
    g = inputs.geometry("batch1k", nsf=1)
    g.grid_n = (40, 36, 44)
    masks = []
    rng = np.random.default_rng(5)
    lrs = []
    specs = [((0, 0, 0), (1, 1, 1), "all", 3), ((3, 4, 5), (5, 2, 7), "none", 0),
             ((10, 8, 6), (6, 5, 4), "random", 16), ((0, 20, 30), (9, 7, 8), "random", 8),
             ((25, 25, 30), (14, 11, 13), "all", 2)]
    for lo, dims, fine, ext in specs:
        m = rng.random((dims[2], dims[1], dims[0])) < 0.8
        m.flat[0] = True
        fm = {"all": m, "none": np.zeros_like(m), "random": m & (rng.random(m.shape) < 0.5)}[fine]
        olo = [max(0, lo[a] - ext) for a in range(3)]
        ohi = [min(g.grid_n[a] - 1, lo[a] + dims[a] - 1 + ext) for a in range(3)]
        om = rng.random((ohi[2] - olo[2] + 1, ohi[1] - olo[1] + 1, ohi[0] - olo[0] + 1)) < 0.9
        ofm = om & (rng.random(om.shape) < 0.6)
        lrs.append(LR.Locreg(lo=lo, dims=dims, ext=ext, cseg=LR.segments_from_mask(m, lo),
                             fseg=LR.segments_from_mask(fm, lo),
                             ocseg=LR.segments_from_mask(om, olo),
                             ofseg=LR.segments_from_mask(ofm, olo)))
    g.centers = np.zeros((len(lrs), 3))
    g.envelope_sigma = np.full(len(lrs), 100.0)
    g.domain_lo = np.zeros(3)
    g.domain_hi = np.array(g.grid_n) * g.h
    case = Case(g, lrs, normalize=False)
    _, _, out, ek, ep = case.run(torch.float64)
    for k in range(len(lrs)):
        ref, rk, rp = case.oracle(k)
        assert rel_err(out[case.out_slice(k)], ref) < 1e-12, k
        assert abs(ek[k] - rk) <= 1e-12 * max(1.0, abs(rk)), k


def _one_point_segments(seg):
    """The same points as one-point segments: segments may touch, so a row
    then holds as many runs as points."""
    out = [(x, x, s[2], s[3]) for s in seg for x in range(int(s[0]), int(s[1]) + 1)]
    return np.array(out, dtype=np.int64).reshape(-1, 4)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_output_rows_with_many_runs(dtype, tol):
    """Rows of 18-24 points (several 16-point windows of the x analysis
    pass) whose patterns hold many runs: random masks, and for every other
    function the same masks as one-point segments, so that a window meets
    up to 16 runs of a row (the most it can).  Dense and sparse output
    masks, ext 2 and 3."""
    _print(f"case: output rows with many runs, {dtype}")
    g = inputs.geometry("batch1k", nsf=1)
    g.grid_n = (56, 24, 24)
    rng = np.random.default_rng(29)
    lrs = []
    for k in range(4):
        lo = (int(rng.integers(6, 10)), int(rng.integers(6, 9)), int(rng.integers(6, 9)))
        dims = (int(rng.integers(18, 25)), int(rng.integers(3, 6)), int(rng.integers(3, 6)))
        ext = 2 if k % 2 == 0 else 3
        m = rng.random((dims[2], dims[1], dims[0])) < 0.7
        m.flat[0] = True
        fm = m & (rng.random(m.shape) < 0.6)
        olo = [lo[a] - ext for a in range(3)]
        oshape = (dims[2] + 2 * ext, dims[1] + 2 * ext, dims[0] + 2 * ext)
        om = rng.random(oshape) < (0.95 if k < 2 else 0.5)
        ofm = om & (rng.random(oshape) < 0.8)
        segs = [LR.segments_from_mask(m, lo), LR.segments_from_mask(fm, lo),
                LR.segments_from_mask(om, olo), LR.segments_from_mask(ofm, olo)]
        if k % 2 == 1:
            segs = [_one_point_segments(s) for s in segs]
        lrs.append(LR.Locreg(lo=lo, dims=dims, ext=ext, cseg=segs[0], fseg=segs[1],
                             ocseg=segs[2], ofseg=segs[3]))
    g.centers = np.zeros((len(lrs), 3))
    g.envelope_sigma = np.full(len(lrs), 100.0)
    g.domain_lo = np.zeros(3)
    g.domain_hi = np.array(g.grid_n) * g.h
    case = Case(g, lrs, normalize=False)
    dt = torch.float64 if dtype == "f64" else torch.float32
    _, _, out, ek, _ = case.run(dt)
    for k in range(len(lrs)):
        ref, rk, _ = case.oracle(k)
        assert rel_err(out[case.out_slice(k)], ref) < tol, k
        if dtype == "f64":
            assert abs(ek[k] - rk) <= 1e-12 * max(1.0, abs(rk)), k


def test_wide_flat_box_fp64():
    """A 70 x 70 x 2 box in FP64: its x-y plane (39.8 KB) leaves room in the
    unpack stage for one component per block only, and its 74-point output
    rows span five windows of the x analysis pass."""
    _print("case: wide flat box, f64")
    g = inputs.geometry("batch1k", nsf=1)
    g.grid_n = (80, 80, 12)
    rng = np.random.default_rng(31)
    lo, dims, ext = (5, 5, 5), (70, 70, 2), 2
    m = rng.random((dims[2], dims[1], dims[0])) < 0.8
    m.flat[0] = True
    fm = m & (rng.random(m.shape) < 0.3)
    olo = [lo[a] - ext for a in range(3)]
    oshape = (dims[2] + 2 * ext, dims[1] + 2 * ext, dims[0] + 2 * ext)
    om = rng.random(oshape) < 0.85
    ofm = om & (rng.random(oshape) < 0.3)
    lrs = [LR.Locreg(lo=lo, dims=dims, ext=ext, cseg=LR.segments_from_mask(m, lo),
                     fseg=LR.segments_from_mask(fm, lo), ocseg=LR.segments_from_mask(om, olo),
                     ofseg=LR.segments_from_mask(ofm, olo))]
    g.centers = np.zeros((1, 3))
    g.envelope_sigma = np.full(1, 100.0)
    g.domain_lo = np.zeros(3)
    g.domain_hi = np.array(g.grid_n) * g.h
    case = Case(g, lrs, normalize=False)
    _, _, out, ek, _ = case.run(torch.float64)
    ref, rk, _ = case.oracle(0)
    assert rel_err(out[case.out_slice(0)], ref) < 1e-12
    assert abs(ek[0] - rk) <= 1e-12 * max(1.0, abs(rk))


def test_chunked_plan_matches_single_chunk_bitwise(spheres):
    _print("case: chunked workspace")
    plan1, _, out1, ek1, ep1 = spheres.run(torch.float64)
    plan2, _, out2, ek2, ep2 = spheres.run(torch.float64, max_workspace=1)
    assert plan2.info["chunks"] == len(spheres.lrs)
    assert np.array_equal(out1, out2) and np.array_equal(ek1, ek2) and np.array_equal(ep1, ep2)


def test_function_alone_equals_function_in_batch(spheres):
    """Batch composition changes no function's result (bitwise)."""
    _print("case: alone vs batch")
    _, _, out, ek, ep = spheres.run(torch.float32)
    k = 3
    alone = Case(spheres.g, [spheres.lrs[k]])
    alone.coefs = [spheres.coefs[k]]
    alone.psi = spheres.coefs[k]
    _, _, out1, ek1, ep1 = alone.run(torch.float32)
    assert np.array_equal(out1, out[spheres.out_slice(k)])
    assert ek1[0] == ek[k] and ep1[0] == ep[k]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sparse_overlap_and_hamiltonian(spheres, dtype):
    """Pattern bit-exact; values against the oracle's S and H (the oracle's H
    uses the oracle's own H|phi>)."""
    _print(f"case: sparse S/H {dtype}")
    dt = torch.float64 if dtype == "f64" else torch.float32
    plan, psi, out, _, _ = spheres.run(dt)
    hpsi = torch.tensor(out, dtype=dt, device="cuda")
    n = len(spheres.lrs)
    ohs = [spheres.oracle(k)[0] for k in range(n)]
    for ket_out in (False, True):
        rowptr, col, val = W.sparse_overlap(plan, psi, hpsi if ket_out else psi, ket_out)
        torch.cuda.synchronize()
        kets = ohs if ket_out else spheres.coefs
        rp, cl, vv = SP.matrix(spheres.lrs, spheres.coefs, kets, ket_out)
        assert np.array_equal(rowptr.cpu().numpy(), rp)
        assert np.array_equal(col.cpu().numpy(), cl)
        v = val.cpu().numpy()
        rtol = 1e-12 if dtype == "f64" else 1e-5
        for a in range(n):
            for j in range(rp[a], rp[a + 1]):
                b = cl[j]
                scale = np.linalg.norm(spheres.coefs[a]) * np.linalg.norm(kets[b])
                assert abs(v[j] - vv[j]) <= rtol * scale, (a, b, v[j], vv[j])
        if not ket_out:
            for a in range(n):
                diag = v[rp[a] + list(cl[rp[a]:rp[a + 1]]).index(a)]
                assert abs(diag - 1.0) < (1e-13 if dtype == "f64" else 1e-6)
        # a second call starts from cleared partials: bitwise the same values
        _, _, val2 = W.sparse_overlap(plan, psi, hpsi if ket_out else psi, ket_out)
        torch.cuda.synchronize()
        assert np.array_equal(val2.cpu().numpy(), v)
        if not ket_out:
            # S with bra == ket sums each pair once and mirrors it; a copy of
            # psi as the ket takes every pair: the same bits
            _, _, val3 = W.sparse_overlap(plan, psi, psi.clone(), False)
            torch.cuda.synchronize()
            assert np.array_equal(val3.cpu().numpy(), v)


def test_repeat_runs_bitwise_deterministic(spheres):
    _print("case: determinism")
    _, _, o1, e1, p1 = spheres.run(torch.float32)
    _, _, o2, e2, p2 = spheres.run(torch.float32)
    assert np.array_equal(o1, o2) and np.array_equal(e1, e2) and np.array_equal(p1, p2)


def test_library_segments_feed_identical_results():
    """Segments built by the library (wvl_build_locregs) equal the oracle's."""
    _print("case: library-built locregs")
    g = inputs.geometry("batch1k", nsf=40)
    lr, segs = W.build_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
    rec, oseg = to_abi(LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext))
    assert np.array_equal(segs, oseg)
    assert np.array_equal(lr["coef_off"], rec["coef_off"])


def test_sparse_on_rows_with_several_runs():
    """Random-mask patterns: rows hold several runs, so both phases of the
    sparse kernel (kept first run, lane-local further runs) are exercised."""
    _print("case: sparse S/H, multi-run rows")
    rng = np.random.default_rng(21)
    g = inputs.geometry("batch1k", nsf=1)
    g.grid_n = (30, 30, 30)
    lrs = []
    for k in range(5):
        lo = tuple(int(v) for v in rng.integers(6, 12, 3))
        dims = tuple(int(v) for v in rng.integers(5, 9, 3))
        ext = 2
        m = rng.random((dims[2], dims[1], dims[0])) < 0.55
        m.flat[0] = True
        fm = m & (rng.random(m.shape) < 0.5)
        olo = [lo[a] - ext for a in range(3)]
        om = rng.random((dims[2] + 2 * ext, dims[1] + 2 * ext, dims[0] + 2 * ext)) < 0.6
        ofm = om & (rng.random(om.shape) < 0.5)
        lrs.append(LR.Locreg(lo=lo, dims=dims, ext=ext, cseg=LR.segments_from_mask(m, lo),
                             fseg=LR.segments_from_mask(fm, lo),
                             ocseg=LR.segments_from_mask(om, olo),
                             ofseg=LR.segments_from_mask(ofm, olo)))
    g.centers = np.zeros((len(lrs), 3))
    g.envelope_sigma = np.full(len(lrs), 100.0)
    g.domain_lo = np.zeros(3)
    g.domain_hi = np.array(g.grid_n) * g.h
    case = Case(g, lrs, normalize=False)
    plan, psi, out, _, _ = case.run(torch.float64)
    hpsi = torch.tensor(out, dtype=torch.float64, device="cuda")
    ohs = [case.oracle(k)[0] for k in range(len(lrs))]
    for ket_out in (False, True):
        rowptr, col, val = W.sparse_overlap(plan, psi, hpsi if ket_out else psi, ket_out)
        torch.cuda.synchronize()
        kets = ohs if ket_out else case.coefs
        rp, cl, vv = SP.matrix(lrs, case.coefs, kets, ket_out)
        assert np.array_equal(rowptr.cpu().numpy(), rp)
        assert np.array_equal(col.cpu().numpy(), cl)
        v = val.cpu().numpy()
        for a in range(len(lrs)):
            for j in range(rp[a], rp[a + 1]):
                scale = np.linalg.norm(case.coefs[a]) * np.linalg.norm(kets[cl[j]])
                assert abs(v[j] - vv[j]) <= 1e-12 * scale, (a, cl[j])


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_update_step(spheres, dtype, tol):
    """wvl_update against the oracle's step, with the oracle's own H phi and
    H_aa: per-function relative L2 error of the updated coefficients."""
    from oracle import update as U
    _print(f"case: update step {dtype}")
    dt = torch.float64 if dtype == "f64" else torch.float32
    plan, psi, out, _, _ = spheres.run(dt)
    hpsi = torch.tensor(out, dtype=dt, device="cuda")
    _, _, hv = W.sparse_overlap(plan, psi, hpsi, True)
    n = len(spheres.lrs)
    ohs = [spheres.oracle(k)[0] for k in range(n)]
    rp, cl, ov = SP.matrix(spheres.lrs, spheres.coefs, ohs, True)
    eta = 0.01
    new = psi.clone()
    W.update(plan, new, hpsi, hv, eta)
    torch.cuda.synchronize()
    got = new.cpu().numpy()
    for k in range(n):
        row = list(cl[rp[k]:rp[k + 1]])
        h_aa = ov[rp[k] + row.index(k)]
        want = U.update(spheres.lrs[k], spheres.coefs[k], ohs[k], h_aa, eta)
        r = spheres.rec[k]
        sl = slice(int(r["coef_off"]), int(r["coef_off"]) + int(r["n_c"]) + 7 * int(r["n_f"]))
        assert rel_err(got[sl], want) < tol, k


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_confining_potential(spheres, dtype, tol):
    """wvl_apply_local_ham_conf against the oracle with a |r - R|^4 added to
    the potential of each function (own prefactor, own centre)."""
    _print(f"case: confinement {dtype}")
    dt = torch.float64 if dtype == "f64" else torch.float32
    n = len(spheres.lrs)
    a = np.linspace(0.004, 0.05, n)
    a[1] = 0.0                                  # one function without confinement
    ctx = W.Context(spheres.g.h, spheres.g.grid_n)
    plan = W.Plan(ctx, spheres.rec, spheres.segs)
    psi = torch.tensor(spheres.psi, dtype=dt, device="cuda")
    pot = torch.tensor(spheres.pot, dtype=dt, device="cuda")
    out = torch.zeros(plan.info["out_coefs"], dtype=dt, device="cuda")
    ek = torch.zeros(n, dtype=torch.float64, device="cuda")
    ep = torch.zeros_like(ek)
    conf = torch.tensor(a, dtype=torch.float64, device="cuda")
    W.apply_local_ham(plan, psi, pot, out, ek, ep, conf=conf)
    torch.cuda.synchronize()
    got, gek, gep = out.cpu().numpy(), ek.cpu().numpy(), ep.cpu().numpy()
    for k in range(n):
        oh, oek, oep = Hm.apply_local_ham(spheres.lrs[k], spheres.coefs[k], spheres.pot,
                                          spheres.g.h, conf=float(a[k]))
        assert rel_err(got[spheres.out_slice(k)], oh) < tol, k
        etol = 1e-12 * max(1.0, abs(oep)) if dtype == "f64" else 1e-6
        assert abs(gep[k] - oep) <= etol, (k, gep[k], oep)
        assert abs(gek[k] - oek) <= (1e-12 * max(1.0, abs(oek)) if dtype == "f64" else 1e-6)


@pytest.mark.parametrize("dtype,tol,conf", [("f64", 1e-12, True), ("f64", 1e-12, False),
                                            ("f32", 1e-5, True)])
def test_preconditioner(spheres, dtype, tol, conf):
    """wvl_precondition (5 conjugate-gradient steps) against the oracle's
    steps, to the apply's bounds (FP64 1e-12, FP32 1e-5 relative).  Each step
    applies the operator once (relative error ~1e-15 in FP64) and forms its
    coefficients from dot products in double; over five steps of a
    well-conditioned operator (kinetic plus a positive shift) the error
    grows by a small factor: measured 7.8e-16 (FP64), 9.4e-8 (FP32)."""
    from oracle import precond as PC
    _print(f"case: preconditioner {dtype} conf={conf}")
    dt = torch.float64 if dtype == "f64" else torch.float32
    n = len(spheres.lrs)
    ctx = W.Context(spheres.g.h, spheres.g.grid_n)
    plan = W.Plan(ctx, spheres.rec, spheres.segs)
    rng = np.random.default_rng(41)
    g = np.concatenate([rng.standard_normal(c.size) for c in spheres.coefs])
    eps = -0.3 - 0.1 * np.arange(n, dtype=np.float64)
    eps[2] = 0.25                                   # taken as 0
    a = np.linspace(0.01, 0.04, n) if conf else np.zeros(n)
    gt = torch.tensor(g, dtype=dt, device="cuda")
    x = torch.zeros_like(gt)
    W.precondition(plan, gt, torch.tensor(eps, device="cuda"), 5, x,
                   conf=torch.tensor(a, device="cuda") if conf else None)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    off = 0
    errs = []
    for k in range(n):
        m = spheres.coefs[k].size
        want = PC.precondition(spheres.lrs[k], g[off:off + m], spheres.g.h, float(a[k]),
                               float(eps[k]), 5)
        errs.append(rel_err(got[off:off + m], want))
        off += m
    _print(f"  worst relative error {max(errs):.2e}")
    for k, e in enumerate(errs):
        assert e < tol, (k, e)
