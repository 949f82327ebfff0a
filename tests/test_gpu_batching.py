"""Batching of uneven boxes: captured graphs and the autotuner, through the C ABI.

A graph replays exactly the eager sequence (bitwise), also when replayed
several times with other device work in between.  A change of bin count only
changes how functions are grouped into launches, so every result stays
bitwise identical; the matrix-core form of the kinetic z part sums in
another order (FP64 1e-12, FP32 1e-5 relative).  A graph captured on the old
layout is refused, and capturing and destroying many graphs does not hold
device memory."""
import numpy as np
import pytest

import inputs
from oracle import locreg as LR
from tests.abi_helpers import rel_err
from tests.test_gpu_parity import Case, _print

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1401_7441_amd as W


def _mixed_case(nsf=10, seed=5):
    """Functions whose boxes differ a lot in size (radii 1.3 to 4.6 bohr)."""
    g = inputs.geometry("batch1k", nsf=nsf, seed_offset=seed)
    rng = np.random.default_rng(1234 + seed)
    g.centers[:] = g.centers.mean(0) + rng.uniform(-5.0, 5.0, (nsf, 3))
    g.radii[:] = np.linspace(1.3, 4.6, nsf)[rng.permutation(nsf)]
    g.fine_radii[:] = np.minimum(1.5, g.radii)
    g.envelope_sigma[:] = g.radii / 2
    lrs = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, 8)
    return Case(g, lrs)


@pytest.fixture(scope="module")
def mixed():
    return _mixed_case()


def _buffers(case, plan, dtype):
    psi = torch.tensor(case.psi, dtype=dtype, device="cuda")
    pot = torch.tensor(case.pot, dtype=dtype, device="cuda")
    out = torch.zeros(plan.info["out_coefs"], dtype=dtype, device="cuda")
    ek = torch.zeros(len(case.lrs), dtype=torch.float64, device="cuda")
    ep = torch.zeros_like(ek)
    ws = plan.new_workspace(dtype)
    return psi, pot, out, ek, ep, ws


def _eager_step(plan, psi, pot, out, ek, ep, ws):
    W.apply_local_ham(plan, psi, pot, out, ek, ep, workspace=ws)
    _, _, s = W.sparse_overlap(plan, psi, psi, False)
    _, _, h = W.sparse_overlap(plan, psi, out, True)
    torch.cuda.synchronize()
    return [t.cpu().numpy().copy() for t in (out, ek, ep, s, h)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_graph_replays_match_eager_step(mixed, dtype):
    _print(f"case: graph replay vs eager, {dtype}")
    dt = torch.float32 if dtype == "f32" else torch.float64
    ctx = W.Context(mixed.g.h, mixed.g.grid_n)
    plan = W.Plan(ctx, mixed.rec, mixed.segs)
    bufs = _buffers(mixed, plan, dt)
    ref = _eager_step(plan, *bufs)
    psi, pot, _, _, _, ws = bufs
    out = torch.zeros_like(bufs[2])
    ek = torch.zeros_like(bufs[3])
    ep = torch.zeros_like(ek)
    s_val = torch.zeros(W.sparse_pattern_nnz(plan, False), dtype=torch.float64, device="cuda")
    h_val = torch.zeros(W.sparse_pattern_nnz(plan, True), dtype=torch.float64, device="cuda")
    g = W.Graph(plan, psi, pot, out, ek, ep, workspace=ws, s_val=s_val, h_val=h_val)
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        got = [t.cpu().numpy().copy() for t in (out, ek, ep, s_val, h_val)]
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), f"replay {rep}"
        # other device work between replays, then clear the outputs
        for t in (out, ek, ep, s_val, h_val):
            t.zero_()
        torch.cuda.synchronize()
    g.close()


def test_autotune_keeps_results_and_invalidates_old_graphs(mixed):
    _print("case: autotune")
    ctx = W.Context(mixed.g.h, mixed.g.grid_n)
    plan = W.Plan(ctx, mixed.rec, mixed.segs)
    psi, pot, out, ek, ep, ws = _buffers(mixed, plan, torch.float32)
    ref = _eager_step(plan, psi, pot, out, ek, ep, ws)
    old = W.Graph(plan, psi, pot, out, ek, ep, workspace=ws)
    best, tried = W.autotune(plan, psi, pot, out, ws, reps=1)
    _print("autotune:", best, len(tried), "layouts")
    assert len(tried) >= 4 and best in tried
    assert min(t["ms"] for t in tried) == best["ms"]
    for kin_mfma in sorted({0, best["kin_mfma"]}, reverse=True):
        W.set_schedule(plan, best["nbins"], kin_mfma)
        out.zero_()
        got = _eager_step(plan, psi, pot, out, ek, ep, ws)
        for a, b in zip(ref, got):
            if kin_mfma:
                assert rel_err(b, a) < 1e-5
            else:
                assert np.array_equal(a, b)
    with pytest.raises(W.WvlError):
        old.launch()
    old.close()
    fresh = W.Graph(plan, psi, pot, out, ek, ep, workspace=ws)
    out.zero_()
    fresh.launch()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref[0])
    fresh.close()


def test_many_graphs_hold_no_device_memory(mixed):
    """A serving engine captures one graph per request: 300 captures and
    destroys on one plan (with S/H values, parallel branches) leave the free
    device memory where it was after the first 20."""
    _print("case: 300 graph captures and destroys")
    ctx = W.Context(mixed.g.h, mixed.g.grid_n)
    plan = W.Plan(ctx, mixed.rec, mixed.segs)
    psi, pot, out, ek, ep, ws = _buffers(mixed, plan, torch.float32)
    s_val = torch.zeros(W.sparse_pattern_nnz(plan, False), dtype=torch.float64, device="cuda")
    h_val = torch.zeros(W.sparse_pattern_nnz(plan, True), dtype=torch.float64, device="cuda")
    free = []
    for k in range(300):
        g = W.Graph(plan, psi, pot, out, ek, ep, workspace=ws, s_val=s_val, h_val=h_val)
        g.launch()
        g.close()
        if k in (19, 299):
            torch.cuda.synchronize()
            free.append(torch.cuda.mem_get_info()[0])
    _print(f"  free device memory after 20 and 300 graphs: {free[0] / 2**20:.1f}, "
           f"{free[1] / 2**20:.1f} MiB")
    assert free[0] - free[1] < 16 << 20


def test_mixed_sizes_against_oracle(mixed):
    """Uneven boxes in one batch, each function against the oracle (FP64)."""
    _print("case: mixed sizes vs oracle")
    _, _, out, ek, ep = mixed.run(torch.float64)
    for k in range(len(mixed.lrs)):
        oh, oek, oep = mixed.oracle(k)
        assert rel_err(out[mixed.out_slice(k)], oh) < 1e-12
        assert abs(ek[k] - oek) <= 1e-12 * max(1.0, abs(oek))
        assert abs(ep[k] - oep) <= 1e-12 * max(1.0, abs(oep))


_FIRST_USE_SCRIPT = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import paper_1401_7441_amd as W
from tests.test_gpu_batching import _mixed_case, _buffers
case = _mixed_case(nsf=6, seed=9)
ctx = W.Context(case.g.h, case.g.grid_n)
plan = W.Plan(ctx, case.rec, case.segs)
psi, pot, out, ek, ep, ws = _buffers(case, plan, torch.float32)
g = W.Graph(plan, psi, pot, out, ek, ep, workspace=ws)   # first launch of any kernel
g.launch()
torch.cuda.synchronize()
got = out.cpu().numpy().copy()
out.zero_()
W.apply_local_ham(plan, psi, pot, out, ek, ep, workspace=ws)
torch.cuda.synchronize()
assert np.array_equal(got, out.cpu().numpy())
best, tried = W.autotune(plan, psi, pot, out, ws, reps=1)
print("ok", best, len(tried), flush=True)
"""


def test_capture_as_first_use_in_a_fresh_process():
    """Regression: a graph captured (or autotuned) before any eager launch in
    the process; kernels must be loaded before the capture starts."""
    import os
    import subprocess
    import sys
    _print("case: capture as the first use of the library")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _FIRST_USE_SCRIPT, root], cwd=root,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    assert "ok" in r.stdout
