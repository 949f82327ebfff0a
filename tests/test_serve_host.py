"""Host logic of the request loop (no GPU): admission order and footprints."""
import numpy as np
import pytest

from paper_1401_7441_amd import serve as S


class _R:
    def __init__(self, rid, arrival, footprint):
        self.rid, self.arrival, self.footprint = rid, arrival, footprint


def test_admission_is_in_arrival_order_and_never_overtakes():
    w = [_R(0, 0.0, 50), _R(1, 0.1, 80), _R(2, 0.2, 10), _R(3, 5.0, 1)]
    # the second request does not fit: the third waits behind it
    assert [r.rid for r in S.admissible(w, now=1.0, free=100)] == [0]
    assert [r.rid for r in S.admissible(w, now=1.0, free=130)] == [0, 1]
    assert [r.rid for r in S.admissible(w, now=1.0, free=1000)] == [0, 1, 2]
    # not yet arrived
    assert [r.rid for r in S.admissible(w, now=-1.0, free=1000)] == []
    assert [r.rid for r in S.admissible(w, now=9.0, free=1000)] == [0, 1, 2, 3]


def test_footprint_counts_every_resident_buffer():
    lr = np.zeros(3, dtype=[("n_c", "<i8"), ("n_f", "<i8"), ("on_c", "<i8"), ("on_f", "<i8")])
    lr["n_c"], lr["n_f"], lr["on_c"], lr["on_f"] = 100, 10, 300, 40
    grid = (10, 10, 10)
    nf = 49 ** 3
    want = 4 * (3 * 170 + 3 * 580 + nf) + 1000 + 2 * 20 * 600 * 3 + 64 * 3
    assert S.footprint_bytes(lr, grid, 4, 1000) == want


def test_percentile_interpolates():
    xs = [1.0, 2.0, 3.0, 4.0, 5.0]
    assert S.percentile(xs, 50) == 3.0
    assert S.percentile(xs, 100) == 5.0
    assert abs(S.percentile(xs, 99) - 4.96) < 1e-12


class _FakeEvent:
    def query(self):
        return True


class _FakeActive:
    """Stands in for the device state of a request (no GPU)."""
    def __init__(self, req, dtype, eta, use_graph, max_workspace, stream):
        if req.rid == 1:
            raise ValueError("malformed request")
        self.req, self.bytes, self.done_event = req, 123, None

    def enqueue_step(self):
        self.done_event = _FakeEvent()

    def close(self):
        pass


@pytest.mark.parametrize("workers", [0, 1])
def test_engine_isolates_a_failing_request(monkeypatch, workers):
    monkeypatch.setattr(S, "_Active", _FakeActive)
    reqs = []
    for i in range(3):
        r = S.Request(rid=i, h=0.45, grid_n=(4, 4, 4), locregs=np.zeros(0), segs=None,
                      psi=None, geom=None, pot_params=None)
        reqs.append(r)
    eng = S.Engine.__new__(S.Engine)
    S.Engine.__init__(eng, hbm_budget=10 ** 9, steps=3, streams=[object(), object()],
                      admit_workers=workers)
    monkeypatch.setattr(eng, "_footprint", lambda r: 1000)
    eng.free_device_bytes = lambda: 1 << 40
    done = eng.run(reqs)
    assert sorted(r.rid for r in done) == [0, 2]
    assert [r.rid for r in eng.failed] == [1] and "malformed" in eng.failed[0].error
    assert eng.used == 0 and eng.stream_load == [0, 0] and eng.step_completions == 6


class _TightActive(_FakeActive):
    """Request 1's set-up runs out of device memory while request 0 is
    active (twice: the first try and the retry after the cache release)."""
    tries = 0

    def __init__(self, req, *args):
        if req.rid == 1 and _TightActive.tries < 2:
            _TightActive.tries += 1
            from paper_1401_7441_amd import WVL_ENOMEM, WvlError
            raise WvlError(WVL_ENOMEM, "hipMalloc(1) returned hipErrorOutOfMemory")
        self.req, self.bytes, self.done_event = req, 123, None


@pytest.mark.parametrize("workers", [0, 1])
def test_engine_defers_a_request_that_finds_no_device_memory(monkeypatch, workers):
    """A request whose set-up fails for device memory while another is
    active goes back to the queue (after one retry with the cache released)
    and is admitted when that request retires; nothing fails."""
    monkeypatch.setattr(S, "_Active", _TightActive)
    _TightActive.tries = 0
    reqs = [S.Request(rid=i, h=0.45, grid_n=(4, 4, 4), locregs=np.zeros(0), segs=None,
                      psi=None, geom=None, pot_params=None) for i in range(2)]
    eng = S.Engine.__new__(S.Engine)
    S.Engine.__init__(eng, hbm_budget=10 ** 9, steps=2, streams=[object()],
                      admit_workers=workers)
    monkeypatch.setattr(eng, "_footprint", lambda r: 1000)
    eng.free_device_bytes = lambda: 0          # always below the footprint
    released = []
    eng.release_cache = lambda: released.append(1)
    done = eng.run(reqs)
    assert sorted(r.rid for r in done) == [0, 1] and not eng.failed
    assert eng.deferred == 1 and _TightActive.tries == 2 and len(released) >= 2
    assert eng.used == 0 and eng.stream_load == [0]
