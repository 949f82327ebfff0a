"""Request loop on the GPU: results alone vs in the mix, one serving step
against the oracle, and the per-function baseline against the engine."""
import numpy as np
import pytest

import inputs
from oracle import hamiltonian as Hm
from oracle import locreg as LR
from oracle import sparse as SP
from oracle import update as U
from tests.abi_helpers import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1401_7441_amd import serve as S


def _print(*a):
    print(*a, flush=True)


def _requests(n, nsf, seed):
    return S.make_requests(n, max_nsf=nsf, seed=seed)


def test_each_result_is_the_same_alone_and_in_the_mix():
    _print("case: serving, alone vs mix")
    reqs = _requests(4, 8, seed=11)
    eng = S.Engine(dtype="f32", steps=3, keep_results=True)
    done = {r.rid: r for r in eng.run(reqs)}
    assert sorted(done) == [0, 1, 2, 3] and eng.step_completions == 12
    for r in _requests(4, 8, seed=11):
        alone = S.Engine(dtype="f32", steps=3, keep_results=True)
        a = alone.run([r])[0]
        for key in ("psi", "e_kin", "e_pot", "s_val", "h_val"):
            assert np.array_equal(a.result[key], done[r.rid].result[key]), (r.rid, key)


def test_staggered_arrivals_join_as_memory_frees():
    _print("case: serving, staggered arrivals and a tight budget")
    reqs = _requests(3, 6, seed=12)
    for i, r in enumerate(reqs):
        r.arrival = 0.05 * i
    eng = S.Engine(dtype="f32", steps=2, keep_results=True)
    # budget for two requests at a time: the third waits for memory
    eng.budget = int(1.5 * max(eng._footprint(r) for r in reqs)) + \
        min(eng._footprint(r) for r in reqs)
    done = eng.run(reqs)
    assert len(done) == 3 and all(r.steps_done == 2 for r in done)
    assert all(r.done > r.arrival for r in done)
    ref = S.Engine(dtype="f32", steps=2, keep_results=True).run(_requests(3, 6, seed=12))
    ref = {r.rid: r for r in ref}
    for r in done:
        assert np.array_equal(r.result["psi"], ref[r.rid].result["psi"])


def test_one_serving_step_against_the_oracle():
    """FP64: apply, H values, update of one request, each function against
    the oracle's apply, H_aa and update (relative 1e-12)."""
    _print("case: serving step vs oracle")
    nsf, seed = 5, 13
    req = _requests(1, nsf, seed=seed)[0]
    eng = S.Engine(dtype="f64", steps=1, keep_results=True)
    got = eng.run([req])[0].result
    g = inputs.geometry("serve", nsf=nsf, seed_offset=seed * 100000)
    lrs = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
    off = np.cumsum([0] + [l.n_c + 7 * l.n_f for l in lrs])
    coefs = [req.psi[off[k]:off[k + 1]] for k in range(nsf)]
    pot = req.potential("cpu", torch.float64).numpy()
    ohs = [Hm.apply_local_ham(lrs[k], coefs[k], pot, g.h)[0] for k in range(nsf)]
    rp, cl, hv = SP.matrix(lrs, coefs, ohs, True)
    for k in range(nsf):
        row = list(cl[rp[k]:rp[k + 1]])
        want = U.update(lrs[k], coefs[k], ohs[k], hv[rp[k] + row.index(k)], eng.eta)
        assert rel_err(got["psi"][off[k]:off[k + 1]], want) < 1e-12, k


def test_per_function_baseline_agrees_with_engine():
    _print("case: per-function FP64 baseline vs engine")
    a = S.run_per_function(_requests(1, 5, seed=14), steps=2, keep_results=True)[0]
    b = S.Engine(dtype="f64", steps=2, keep_results=True).run(_requests(1, 5, seed=14))[0]
    assert rel_err(a.result["psi"], b.result["psi"]) < 1e-13


def test_malformed_request_fails_alone():
    """A request whose segment offsets are not running sums is rejected by
    the library at plan creation; it lands in `failed` with the library's
    message, its memory is returned, and the requests around it finish with
    the same results as without it."""
    _print("case: serving, a malformed request among good ones")
    reqs = _requests(3, 6, seed=15)
    bad = reqs[1].fresh()
    bad.rid = 99
    bad.segs = bad.segs.copy()
    bad.segs["off"][1] += 1
    eng = S.Engine(dtype="f32", steps=2, keep_results=True)
    done = {r.rid: r for r in eng.run(reqs + [bad])}
    assert sorted(done) == [0, 1, 2]
    assert [r.rid for r in eng.failed] == [99] and "running sum" in eng.failed[0].error
    assert eng.used == 0 and not eng.active and all(v == 0 for v in eng.stream_load)
    ref = {r.rid: r for r in S.Engine(dtype="f32", steps=2, keep_results=True).run(
        _requests(3, 6, seed=15))}
    for k in done:
        assert np.array_equal(done[k].result["psi"], ref[k].result["psi"])


def test_small_request_is_not_held_back_by_a_large_one():
    """Steps advance per request and set-ups run side by side on worker
    threads: a 20-function request admitted beside a 2,000-function one
    finishes its 5 steps in a fraction of the large one's time, counted from
    admission."""
    _print("case: serving, a small request beside a large one")
    big = S.make_requests(1, nsf=2000, seed=16, fast=True)[0]
    small = S.make_requests(1, nsf=20, seed=17, fast=True)[0]
    small.rid = 1
    eng = S.Engine(dtype="f32", steps=5)
    eng.run([big, small])
    got = {r.rid: r for r in eng.finished}
    assert got[1].nsf == 20 and got[0].nsf == 2000
    small_t = got[1].done - got[1].admitted
    big_t = got[0].done - got[0].admitted
    _print(f"  from admission: small {small_t:.3f} s, large {big_t:.3f} s")
    assert small_t < 0.5 * big_t, (small_t, big_t)
