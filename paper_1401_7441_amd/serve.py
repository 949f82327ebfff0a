"""Request loop: continuous batching of independent systems on one GPU.

Each request is one system of support functions (its own grid, potential,
localization regions and coefficients) that needs `steps` update steps:
local-H apply, overlap and Hamiltonian values on the resident patterns, then
the update psi <- psi - eta (P_L H psi - H_aa psi) (wvl_update).  The compressed
coefficients, H psi, the potential, the plan (keys and patterns) and the
step graph stay on the device across the steps.  This reuse of resident
support functions is what the method relies on between geometry steps and
between neutral and charged runs (paper Sec. VIII).

Scheduling:
  * admission by HBM footprint: a waiting request is admitted, in arrival
    order, as soon as its footprint (coefficients, H psi, potential,
    workspace, patterns) fits in the budget left by the active requests;
    after its plan exists the estimate is replaced by the bytes the request
    actually holds;
  * set-up off the loop: an admitted request's plan, patterns, potential
    and step graph are built on a worker thread while the host goes on
    enqueuing the active requests' steps;
  * continuous batching: every active request runs its steps on its own
    HIP stream, so the kernels of different requests overlap on the device;
    the host polls each request's last step and enqueues its next one as
    soon as it is done, independently of the others (a small request is
    never held back by a large one), retires it after its last step and
    admits waiting requests into the memory it frees;
  * failure isolation: a request whose set-up or step fails (a malformed
    request, an allocation that does not fit) is moved to `failed` with its
    error, its memory is returned, and the others go on;
  * latency = arrival -> completion of the last step (host clock).

The per-function baseline (`run_per_function`) is the plain path: FP64, one
support function per apply (a one-function plan each), no graphs, one
request at a time.

Every step of the path runs in the library's kernels; this module only
schedules them and moves data.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import (Context, Graph, Plan, apply_local_ham, build_locregs, sparse_overlap,
               sparse_pattern_nnz, update)


@dataclasses.dataclass
class Request:
    """One system.  Host inputs (segments, coefficients) are prepared before
    submission; the potential is given by its Gaussian wells (`geom`,
    `pot_params`) and built on the device at admission, where a DFT code
    would produce it."""
    rid: int
    h: float
    grid_n: tuple
    locregs: np.ndarray
    segs: np.ndarray
    psi: np.ndarray
    geom: object
    pot_params: tuple
    arrival: float = 0.0
    # filled by the engine
    admitted: float = math.nan
    done: float = math.nan
    steps_done: int = 0
    footprint: int = 0
    memory_retries: int = 0
    error: str = ""
    result: dict = dataclasses.field(default_factory=dict)

    @property
    def nsf(self):
        return len(self.locregs)

    @property
    def latency(self):
        return self.done - self.arrival

    def potential(self, device, dtype):
        """The global fine-grid potential (torch tensor, z, y, x)."""
        import inputs
        return inputs.potential(self.geom, device=device, dtype=dtype,
                                params=self.pot_params).contiguous()

    def fresh(self, arrival=0.0):
        """A new request on the same inputs (shared host arrays)."""
        return Request(rid=self.rid, h=self.h, grid_n=self.grid_n, locregs=self.locregs,
                       segs=self.segs, psi=self.psi, geom=self.geom, pot_params=self.pot_params,
                       arrival=arrival)


def footprint_bytes(locregs, grid_n, sz, workspace_bytes, nnz_bound=None):
    """Device bytes a request holds while active (before its plan exists the
    workspace size comes from the plan; patterns are bounded by 600 pairs per
    function, each pair 12 bytes of CSR plus 8 of values, for S and H)."""
    n_in = int(np.sum(locregs["n_c"] + 7 * locregs["n_f"]))
    n_out = int(np.sum(locregs["on_c"] + 7 * locregs["on_f"]))
    nf = (2 * grid_n[0] + 29) * (2 * grid_n[1] + 29) * (2 * grid_n[2] + 29)
    nnz = nnz_bound if nnz_bound is not None else 600 * len(locregs)
    return int(sz * (n_in + n_out + nf) + workspace_bytes + 2 * 20 * nnz + 64 * len(locregs))


class _Active:
    """Device state of an admitted request."""

    def __init__(self, req: Request, dtype, eta, use_graph, max_workspace, stream):
        import torch
        self.req = req
        self.stream = stream
        with torch.cuda.stream(self.stream):
            self.ctx = Context(req.h, req.grid_n, stream=self.stream)
            self.plan = Plan(self.ctx, req.locregs, req.segs, max_workspace=max_workspace)
            self.psi = torch.from_numpy(req.psi).to(dtype).to("cuda", non_blocking=True)
            self.pot = req.potential("cuda", dtype)
            self.hpsi = torch.zeros(self.plan.info["out_coefs"], dtype=dtype, device="cuda")
            self.ek = torch.zeros(req.nsf, dtype=torch.float64, device="cuda")
            self.ep = torch.zeros_like(self.ek)
            self.ws = self.plan.new_workspace(dtype)
            self.nnz_s = sparse_pattern_nnz(self.plan, False)
            self.nnz_h = sparse_pattern_nnz(self.plan, True)
            self.s_out = (torch.zeros(req.nsf + 1, dtype=torch.int64, device="cuda"),
                          torch.zeros(max(1, self.nnz_s), dtype=torch.int32, device="cuda"),
                          torch.zeros(max(1, self.nnz_s), dtype=torch.float64, device="cuda"))
            self.h_out = (torch.zeros(req.nsf + 1, dtype=torch.int64, device="cuda"),
                          torch.zeros(max(1, self.nnz_h), dtype=torch.int32, device="cuda"),
                          torch.zeros(max(1, self.nnz_h), dtype=torch.float64, device="cuda"))
            self.s_val, self.h_val = self.s_out[2], self.h_out[2]
        self.eta = eta
        self.graph = None
        self.done_event = None
        if use_graph:
            self.graph = Graph(self.plan, self.psi, self.pot, self.hpsi, self.ek, self.ep,
                               workspace=self.ws, s_val=self.s_val, h_val=self.h_val)
        # device bytes this request holds (the graph's own are small)
        self.bytes = int(sum(t.numel() * t.element_size() for t in
                             (self.psi, self.pot, self.hpsi, self.ek, self.ep, self.ws,
                              *self.s_out, *self.h_out)))
        self.bytes += 24 * (self.nnz_s + self.nnz_h) + 8 * 1024 * req.nsf   # plan patterns, keys

    def enqueue_step(self):
        import torch
        with torch.cuda.stream(self.stream):
            if self.graph is not None:
                self.graph.launch()
            else:
                apply_local_ham(self.plan, self.psi, self.pot, self.hpsi, self.ek, self.ep,
                                workspace=self.ws)
                sparse_overlap(self.plan, self.psi, self.psi, False, out=self.s_out)
                sparse_overlap(self.plan, self.psi, self.hpsi, True, out=self.h_out)
            update(self.plan, self.psi, self.hpsi, self.h_val, self.eta)
            self.done_event = torch.cuda.Event()
            self.done_event.record(self.stream)

    def snapshot(self):
        """Final state to host: psi, energies, S and H values."""
        self.stream.synchronize()
        return {"psi": self.psi.cpu().numpy(), "e_kin": self.ek.cpu().numpy(),
                "e_pot": self.ep.cpu().numpy(),
                "s_val": self.s_val[:self.nnz_s].cpu().numpy(),
                "h_val": self.h_val[:self.nnz_h].cpu().numpy()}

    def close(self):
        self.stream.synchronize()
        if getattr(self, "graph", None) is not None:
            self.graph.close()
        for name in ("plan", "ctx"):
            obj = getattr(self, name, None)
            if obj is not None:
                obj.close()


def _activate(req, dtype, eta, use_graph, max_workspace, stream):
    """_Active(req, ...), releasing whatever was created when it fails."""
    a = _Active.__new__(_Active)
    try:
        a.__init__(req, dtype, eta, use_graph, max_workspace, stream)
    except Exception:
        try:
            a.close()
        except Exception:
            pass
        raise
    return a


class Engine:
    """Continuous-batching engine (see the module docstring)."""

    def __init__(self, dtype="f32", hbm_budget=None, eta=0.01, steps=5, use_graph=True,
                 max_workspace=8 << 30, keep_results=False, n_streams=8, streams=None,
                 admit_workers=2):
        import torch
        # a fixed pool of streams (default priority): requests take the one
        # with the fewest active requests; buffers are allocated on it, so
        # freed memory returns to a stream that stays in use
        self.streams = streams if streams is not None else \
            [torch.cuda.Stream() for _ in range(n_streams)]
        self.stream_load = [0] * len(self.streams)
        self.dtype = torch.float32 if dtype == "f32" else torch.float64
        self.sz = 4 if dtype == "f32" else 8
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.85 * free)
        self.budget = int(hbm_budget)
        self.eta = eta
        self.steps = steps
        self.use_graph = use_graph
        self.max_workspace = int(max_workspace)
        self.keep_results = keep_results
        self.waiting = []
        self.active = []
        self.finished = []
        self.rejected = []       # footprint above the whole budget
        self.failed = []         # set-up or a step raised (req.error holds why)
        self.used = 0
        self.step_completions = 0
        self.sf_steps = 0
        self.held_back = False   # admission waits for a retirement (see _admit)
        # set-up of admitted requests (plan, patterns, potential, graph) runs
        # on worker threads, so the host keeps enqueuing the active requests'
        # steps meanwhile, and a small request's set-up need not wait behind
        # a large one's; 0 workers: set-up inline
        self.admit_workers = admit_workers
        self.setting_up = []     # (request, stream index, future)
        self._pool = None
        # device memory probes (replaceable for host-only tests)
        self.free_device_bytes = lambda: torch.cuda.mem_get_info()[0]
        self.release_cache = torch.cuda.empty_cache
        self.deferred = 0        # admissions put back for lack of device memory

    def _footprint(self, req):
        # the workspace of a plan bounded by max_workspace is at most that bound
        # plus one function's share; estimate it without creating the plan
        ws = min(self.max_workspace + (64 << 20), 16 * (1 << 20) * req.nsf * self.sz // 4)
        return footprint_bytes(req.locregs, req.grid_n, self.sz, ws)

    def submit(self, req: Request):
        req.footprint = self._footprint(req)
        if req.footprint > self.budget:
            self.rejected.append(req)
        else:
            self.waiting.append(req)

    def _now(self):
        return time.perf_counter() - self.t0

    def _release(self, a):
        self.stream_load[a.stream_index] -= 1
        self.used -= a.held
        self.held_back = False

    def _fail(self, req, err, a=None):
        req.error = f"{type(err).__name__}: {err}"
        req.done = self._now()
        if a is not None:
            try:
                a.close()
            except Exception:
                pass
            self._release(a)
        self.failed.append(req)

    def _activate_with_memory(self, r, si):
        """_activate, making room first: device memory that torch's caching
        allocator keeps for the tensors of retired requests is not available
        to the library's own allocations (plans, patterns, graphs), so the
        cache is released when the device's free memory is below the
        request's footprint, and once more after an allocation failure."""
        if self.free_device_bytes() < r.footprint + (1 << 30):
            self.release_cache()
        try:
            return _activate(r, self.dtype, self.eta, self.use_graph, self.max_workspace,
                             self.streams[si])
        except Exception as err:
            if not _out_of_memory(err):
                raise
        self.release_cache()
        return _activate(r, self.dtype, self.eta, self.use_graph, self.max_workspace,
                         self.streams[si])

    def _admit(self):
        """Admits every waiting request that has arrived and fits, in order;
        each starts its first step at once.  A request that fits the budget
        but finds too little device memory (fragmentation the accounting
        does not see) goes back to the head of the queue while other
        requests are active, and is retried when one of them retires."""
        if self.held_back:
            return
        for r in admissible(self.waiting, self._now(), self.budget - self.used):
            self.waiting.remove(r)
            r.admitted = self._now()
            si = min(range(len(self.streams)), key=lambda i: self.stream_load[i])
            self.stream_load[si] += 1
            self.used += r.footprint
            if self.admit_workers:
                if self._pool is None:
                    from concurrent.futures import ThreadPoolExecutor
                    self._pool = ThreadPoolExecutor(self.admit_workers)
                self.setting_up.append((r, si, self._pool.submit(self._activate_with_memory,
                                                                 r, si)))
                continue
            try:
                act = self._activate_with_memory(r, si)
            except Exception as err:            # malformed request, no memory, ...
                if not self._setup_failed(r, si, err):
                    return
                continue
            self._start(act, si)

    def _setup_failed(self, r, si, err):
        """Undoes an admission whose set-up raised: the request goes back to
        the queue when it found no device memory while others are active
        (returns False: stop admitting), else it fails (returns True)."""
        self.stream_load[si] -= 1
        self.used -= r.footprint
        busy = bool(self.active or self.setting_up)
        # with a worker, the requests it ran beside may have retired since
        if _out_of_memory(err) and (busy or r.memory_retries < 1):
            r.memory_retries += 0 if busy else 1
            r.admitted = math.nan
            self.waiting.append(r)
            self.held_back = busy
            self.deferred += 1
            return False
        self._fail(r, err)
        return True

    def _start(self, act, si):
        act.stream_index = si
        # what the request actually holds replaces the estimate
        act.held = int(getattr(act, "bytes", act.req.footprint))
        self.used += act.held - act.req.footprint
        self.active.append(act)
        self._step(act)

    def _collect(self):
        """Starts the requests whose set-up has finished; returns how many."""
        n = 0
        for item in list(self.setting_up):
            r, si, fut = item
            if not fut.done():
                continue
            self.setting_up.remove(item)
            n += 1
            try:
                act = fut.result()
            except Exception as err:
                self._setup_failed(r, si, err)
                continue
            self._start(act, si)
        return n

    def _step(self, a):
        try:
            a.enqueue_step()
        except Exception as err:
            self.active.remove(a)
            self._fail(a.req, err, a)

    def poll(self):
        """One pass over the active requests: each whose last step is done
        counts it, then retires or enqueues its next step.  Returns the
        number of steps completed in this pass."""
        n = 0
        for a in list(self.active):
            if not a.done_event.query():
                continue
            n += 1
            self.step_completions += 1
            a.req.steps_done += 1
            self.sf_steps += a.req.nsf
            if a.req.steps_done < self.steps:
                self._step(a)
                continue
            a.req.done = self._now()
            self.active.remove(a)
            try:
                if self.keep_results:
                    a.req.result = a.snapshot()
                a.close()
            except Exception as err:
                self._release(a)
                a.req.error = f"{type(err).__name__}: {err}"
                self.failed.append(a.req)
                continue
            self._release(a)
            self.finished.append(a.req)
        return n

    def run(self, requests, t0=None, poll_s=50e-6, progress=None, every=100):
        """Serve `requests` (their `arrival` times in seconds from now) until
        all are finished or failed.  Returns the finished requests.
        `progress(ended, total, seconds)` is called each time another
        `every` requests have ended (finished or failed)."""
        self.t0 = time.perf_counter() if t0 is None else t0
        for r in requests:
            self.submit(r)
        total = len(self.waiting)
        reported = 0
        while self.waiting or self.active or self.setting_up:
            self._admit()
            if self._collect() + self.poll():
                ended = len(self.finished) + len(self.failed)
                if progress is not None and ended - reported >= every:
                    reported = ended
                    progress(ended, total, self._now())
                continue
            if self.active or self.setting_up:
                time.sleep(poll_s)
            elif self.waiting:
                # idle until the next arrival (or until memory frees, which
                # cannot happen with nothing active: the head does not fit)
                nxt = min(r.arrival for r in self.waiting)
                delay = nxt - self._now()
                if delay > 0:
                    time.sleep(min(delay, 0.05))
                elif not admissible(self.waiting, self._now(), self.budget - self.used):
                    # the head of the queue can never fit: fail it
                    head = min(self.waiting, key=lambda r: (r.arrival, r.rid))
                    self.waiting.remove(head)
                    self._fail(head, MemoryError("footprint above the free budget"))
        if self._pool is not None:
            self._pool.shutdown(wait=True)
            self._pool = None
        return self.finished


def _out_of_memory(err):
    """Whether an exception is a device allocation failure (the library's
    WVL_ENOMEM or torch's out-of-memory error)."""
    from . import WVL_ENOMEM, WvlError
    if isinstance(err, WvlError):
        return err.status == WVL_ENOMEM
    return type(err).__name__ == "OutOfMemoryError" or "out of memory" in str(err)


def admissible(waiting, now, free):
    """Requests to admit now: those that have arrived, in arrival order, as
    long as their footprints fit in `free` bytes; the first one that does
    not fit stops the scan (no overtaking, so a large request is never
    starved by smaller ones behind it)."""
    out = []
    for r in sorted(waiting, key=lambda r: (r.arrival, r.rid)):
        if r.arrival > now or r.footprint > free:
            break
        out.append(r)
        free -= r.footprint
    return out


def run_per_function(requests, eta=0.01, steps=5, keep_results=False):
    """The plain baseline: FP64, each support function applied alone (a
    one-function plan per function), no graphs, requests served one at a
    time in arrival order.  Returns the requests with done / latency set."""
    import torch
    t0 = time.perf_counter()
    out = []
    for req in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if now < req.arrival:
            time.sleep(req.arrival - now)
        ctx = Context(req.h, req.grid_n)
        full = Plan(ctx, req.locregs, req.segs)
        psi = torch.from_numpy(req.psi).to(torch.float64).cuda()
        pot = req.potential("cuda", torch.float64)
        hpsi = torch.zeros(full.info["out_coefs"], dtype=torch.float64, device="cuda")
        singles = []
        for k in range(req.nsf):
            one = req.locregs[k:k + 1].copy()
            sg = req.segs
            # a one-function plan over the same segment array and offsets
            singles.append(_single_plan(ctx, one, sg))
        for _ in range(steps):
            for k, (plan1, in_off, out_off) in enumerate(singles):
                n_in, n_out = plan1.info["in_coefs"], plan1.info["out_coefs"]
                o = torch.zeros(n_out, dtype=torch.float64, device="cuda")
                apply_local_ham(plan1, psi[in_off:in_off + n_in].contiguous(), pot, o)
                hpsi[out_off:out_off + n_out] = o
            sparse_overlap(full, psi, psi, False)
            _, _, hv = sparse_overlap(full, psi, hpsi, True)
            update(full, psi, hpsi, hv, eta)
        torch.cuda.synchronize()
        req.done = time.perf_counter() - t0
        req.steps_done = steps
        if keep_results:
            req.result = {"psi": psi.cpu().numpy()}
        for p, _, _ in singles:
            p.close()
        full.close()
        ctx.close()
        out.append(req)
    return out


def _single_plan(ctx, one, segs):
    """A plan for one function with its own segments and coefficients at
    offset 0 (the function's own slices of the request's buffers)."""
    in_off, out_off = int(one["coef_off"][0]), int(one["ocoef_off"][0])
    parts, base = [], 0
    for key, cnt in (("seg_c", "nseg_c"), ("seg_f", "nseg_f"), ("oseg_c", "noseg_c"),
                     ("oseg_f", "noseg_f")):
        a, n = int(one[key][0]), int(one[cnt][0])
        parts.append(segs[a:a + n])
        one[key] = base
        base += n
    one["coef_off"] = 0
    one["ocoef_off"] = 0
    return Plan(ctx, one, np.concatenate(parts)), in_off, out_off


def make_requests(n, dtype_sz=4, rate=None, seed=0, max_nsf=None, ngauss=32, fast=False,
                  nsf=None):
    """`n` serving requests drawn as the serving workload (systems of 50-4000
    support functions, log-uniform) with Poisson arrivals at `rate` per
    second (all at t = 0 when rate is None).  Host inputs only.  With
    `fast`, each request's coefficients are N(0, 1/n_coef) from one stream
    per request instead of the per-function enveloped draws (the work done
    does not depend on the values).  `nsf` fixes the size, `max_nsf` caps
    the drawn one."""
    import inputs
    rng = np.random.default_rng(7000 + seed)
    t = 0.0
    reqs = []
    for i in range(n):
        g = inputs.geometry("serve", nsf=nsf, seed_offset=seed * 100000 + i)
        if max_nsf is not None and len(g.radii) > max_nsf:
            g = inputs.geometry("serve", nsf=max_nsf, seed_offset=seed * 100000 + i)
        lr, segs = build_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
        if fast:
            n_in = int(np.sum(lr["n_c"] + 7 * lr["n_f"]))
            psi = inputs.flat_coefficients(g, n_in, seed=seed * 100000 + i)
        else:
            psi = np.concatenate([
                inputs.coefficients(g, k, _pts(segs, lr[k], "c"), _pts(segs, lr[k], "f"))
                for k in range(len(lr))])
        params = inputs.potential_params(g, ngauss=min(ngauss, len(lr)))
        if rate is not None:
            t += rng.exponential(1.0 / rate)
        reqs.append(Request(rid=i, h=g.h, grid_n=tuple(g.grid_n), locregs=lr, segs=segs,
                            psi=psi, geom=g, pot_params=params,
                            arrival=t if rate is not None else 0.0))
    return reqs


def _pts(segs, r, kind):
    a = int(r["seg_c" if kind == "c" else "seg_f"])
    n = int(r["nseg_c" if kind == "c" else "nseg_f"])
    rows = segs[a:a + n]
    if n == 0:
        return np.zeros((0, 3), np.int64)
    return np.concatenate([np.stack([np.arange(s["i1s"], s["i1e"] + 1),
                                     np.full(s["i1e"] - s["i1s"] + 1, s["i2"]),
                                     np.full(s["i1e"] - s["i1s"] + 1, s["i3"])], axis=1)
                           for s in rows])


# request sizes (support functions) of the per-bucket latencies
SIZE_BUCKETS = ((50, 200), (200, 1000), (1000, 4001))


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return math.nan
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def _trace(pool, n, rate, seed):
    """n requests drawn uniformly from the prepared systems of `pool`, with
    Poisson arrivals at `rate` per second (all at t = 0 when rate is None);
    each is a fresh request on its system's host inputs."""
    rng = np.random.default_rng(9000 + seed)
    pick = rng.integers(0, len(pool), n)
    t = np.cumsum(rng.exponential(1.0 / rate, n)) if rate else np.zeros(n)
    out = []
    for j, (i, a) in enumerate(zip(pick, t)):
        r = pool[int(i)].fresh(float(a))
        r.rid = j
        out.append(r)
    return out


def _latencies(done):
    lat = [r.latency for r in done]
    buckets = {}
    for lo, hi in SIZE_BUCKETS:
        bl = [r.latency for r in done if lo <= r.nsf < hi]
        buckets[f"{lo}-{hi - 1}"] = {"requests": len(bl), "p50_s": percentile(bl, 50),
                                     "p99_s": percentile(bl, 99)}
    return lat, buckets


def benchmark(n_requests=24, load=0.8, dtype="f32", steps=5, seed=1, baseline_requests=4,
              log=print, loads=(0.5, 0.95), pool_size=None, n_other=None, n_saturated=None,
              progress_every=100, mu=None):
    """Serving measurement on requests drawn from a pool of `pool_size`
    prepared systems (sizes log-uniform, as the serving workload; by default
    one system per request): (1) saturated throughput with `n_saturated`
    requests queued at t = 0; (2) Poisson arrivals at `load` x that request
    rate, `n_requests` of them, p50 and p99 latency overall and by size;
    (3) the same at each of `loads` with `n_other` requests; (4) the
    per-function FP64 baseline: the first `baseline_requests` requests of
    the `load` trace, each served alone (its service time: the plain path
    cannot keep up with the offered rate, so under that arrival stream its
    queue, and its latency, grow without bound).  A log line is written
    each time another `progress_every` requests of a run have ended.  With
    `mu` (requests/s, from an earlier saturated run on the same pool and
    seed) the saturated run is skipped and the loads are fractions of `mu`.
    Returns a dict of the figures."""
    import torch
    pool_size = pool_size or n_requests
    n_other = n_other or n_requests
    n_saturated = n_saturated or n_requests
    t0 = time.perf_counter()
    pool = make_requests(pool_size, seed=seed, fast=True)
    t_prep = time.perf_counter() - t0
    sizes = [r.nsf for r in pool]
    log(f"serving: pool of {pool_size} systems, {sum(sizes)} functions "
        f"(min {min(sizes)}, median {int(np.median(sizes))}, max {max(sizes)}), "
        f"inputs prepared in {t_prep:.1f} s")
    # warm-up on a small request (kernel loads, allocator)
    Engine(dtype=dtype, steps=1).run(make_requests(1, seed=seed + 99, max_nsf=50, fast=True))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]

    def prog(name):
        return lambda k, n, t: log(f"serving: {name}: {k}/{n} requests ended, {t:.1f} s")

    if mu is None:
        reqs = _trace(pool, n_saturated, None, seed)
        eng = Engine(dtype=dtype, steps=steps)
        t1 = time.perf_counter()
        eng.run(reqs, progress=prog("saturated"), every=progress_every)
        t_sat = time.perf_counter() - t1
        mu = len(eng.finished) / t_sat
        sat = {"requests": n_saturated, "seconds": t_sat, "requests_per_s": mu,
               "sf_steps_per_s": eng.sf_steps / t_sat,
               "step_completions": eng.step_completions, "failed": len(eng.failed),
               "deferred_for_memory": eng.deferred}
        log(f"serving: saturated {t_sat:.2f} s, {mu:.2f} requests/s, "
            f"{eng.sf_steps / t_sat:.0f} support-function steps/s")
        if eng.failed:
            raise RuntimeError(f"serving: request {eng.failed[0].rid} failed: "
                               f"{eng.failed[0].error}")
    else:
        sat = {"requests_per_s": float(mu), "note": "given (earlier saturated run)"}

    def poisson(ld, n):
        rate = ld * mu
        reqs2 = _trace(pool, n, rate, seed + int(100 * ld))
        eng2 = Engine(dtype=dtype, steps=steps)
        t2 = time.perf_counter()
        done = eng2.run(reqs2, progress=prog(f"load {ld}"), every=progress_every)
        t_run = time.perf_counter() - t2
        if eng2.failed:
            raise RuntimeError(f"serving: load {ld}: request {eng2.failed[0].rid} failed: "
                               f"{eng2.failed[0].error}")
        lat, buckets = _latencies(done)
        res = {"requests": n, "offered_requests_per_s": rate, "load": ld, "seconds": t_run,
               "requests_per_s": len(done) / t_run, "sf_steps_per_s": eng2.sf_steps / t_run,
               "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
               "max_s": max(lat), "rejected": len(eng2.rejected), "failed": len(eng2.failed),
               "deferred_for_memory": eng2.deferred, "by_size": buckets}
        log(f"serving: load {ld}, {n} requests: p50 {res['p50_s']:.3f} s, "
            f"p99 {res['p99_s']:.3f} s")
        return res, reqs2, done

    served, trace, done = poisson(load, n_requests)
    others = [poisson(ld, n_other)[0] for ld in loads if ld != load]
    torch.cuda.synchronize()
    # device memory the runs left held (graphs, plans, streams), torch's
    # cache of freed blocks released first on both sides of the difference
    torch.cuda.empty_cache()
    held_mib = (free0 - torch.cuda.mem_get_info()[0]) / 2**20
    base = None
    if baseline_requests:
        svc, sz = [], []
        tb = time.perf_counter()
        for k, r in enumerate(trace[:baseline_requests]):
            one = run_per_function([r.fresh(0.0)], steps=steps)[0]
            svc.append(one.latency)
            sz.append(r.nsf)
            if progress_every and (k + 1) % max(1, progress_every // 10) == 0:
                log(f"serving: per-function baseline: {k + 1}/{baseline_requests} requests")
        eng_lat = {r.rid: r.latency for r in done}
        same = [eng_lat[r.rid] for r in trace[:baseline_requests] if r.rid in eng_lat]
        base = {"requests": baseline_requests, "seconds": time.perf_counter() - tb,
                "service_p50_s": percentile(svc, 50), "service_p99_s": percentile(svc, 99),
                "requests_per_s": len(svc) / sum(svc),
                "offered_requests_per_s": served["offered_requests_per_s"],
                "engine_p50_s_same_requests": percentile(same, 50),
                "engine_p99_s_same_requests": percentile(same, 99),
                "sizes": sz,
                "kind": "FP64, one support function per apply, no graphs, each request "
                        "alone (service time, no queueing)"}
        log(f"serving: per-function FP64 baseline, {baseline_requests} requests alone: "
            f"service p50 {base['service_p50_s']:.3f} s, p99 {base['service_p99_s']:.3f} s, "
            f"{base['requests_per_s']:.3f} requests/s")
    return {"pool": pool_size, "functions_in_pool": sum(sizes), "steps": steps, "dtype": dtype,
            "saturated": sat, "poisson": served,
            "poisson_other_loads": others, "per_function_fp64": base,
            "device_mib_held_after_runs": held_mib,
            "latency_note": "arrival -> end of the last step, host clock; requests drawn "
                            "from the pool's systems"}


def main(argv=None):
    """Serving benchmark from the command line; writes one JSON document."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--requests", type=int, default=1000, help="Poisson requests at --load")
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--loads", type=float, nargs="*", default=[],
                    help="further load levels, --other requests each")
    ap.add_argument("--other", type=int, default=1000)
    ap.add_argument("--saturated", type=int, default=200)
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--baseline", type=int, default=0,
                    help="requests of the trace served alone by the per-function FP64 path")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--progress-every", type=int, default=100)
    ap.add_argument("--mu", type=float, default=None,
                    help="saturated requests/s from an earlier run (skips the saturated run)")
    ap.add_argument("--out", default="-")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    res = benchmark(n_requests=args.requests, load=args.load, dtype=args.dtype,
                    steps=args.steps, seed=args.seed, baseline_requests=args.baseline, log=log,
                    loads=tuple(args.loads), pool_size=args.pool, n_other=args.other,
                    n_saturated=args.saturated, progress_every=args.progress_every,
                    mu=args.mu)
    text = json.dumps(res, indent=1)
    if args.out == "-":
        print(text)
    else:
        with open(args.out, "w") as f:
            f.write(text + "\n")


if __name__ == "__main__":
    main()
