"""Continuous-batching serving loop over many independent filters.

Each monitoring stream is one HiKF filter (its own grid, rays, kernel and
n_c); a request is one assimilation step of one stream (Algorithm
Algorithm_HiKF: predict and correct with that stream's next measurement).
The loop

* keeps every admitted stream's state (x_hat, diag P, the cross-covariance
  C, C_Q, the tree operators' results, the captured step graph) resident in
  HBM, and admits streams by memory: a stream is built (hikf_init) when its
  resident region fits in the HBM budget; when it does not, idle streams
  (nothing queued or running) are evicted, least recently used first, their
  state saved to host memory (hikf_export_checkpoint: x_hat, diag P, C, the
  carried p-space state and the step count) and restored on the next
  admission (hikf_init recomputes the same C_Q, hikf_import_checkpoint puts
  the state back), so a stream's results do not depend on evictions;
* dispatches continuously: it polls the device for finished steps and for
  new arrivals and issues every queued request as soon as its stream has a
  device stream (a slot) — no request waits for others to finish a round.
  A stream keeps one slot while it has steps in flight, so its own steps
  run in order; different streams' steps overlap on the device;
* measures each request from its arrival (host clock) to the moment the
  loop sees its completion event.

Nothing here computes: every step runs in libhikf.so through the C ABI;
this module only decides what runs when, and owns the device memory (torch).
``run_sequential`` is the plain one-filter-at-a-time path on the same
requests, for comparison.
"""

import collections
import time

import numpy as np
import torch

from . import filter as F


class StreamSpec:
    """One monitoring stream: its problem (CSR H on the host, R, kernel) and
    filter options."""

    def __init__(self, dim, n, rowptr, col, val, r_diag, theta=1.0, ell=1.0, gamma=1.0,
                 n_c=4, precision="f32", prior="kernel", sparse=True, psd_guard=False, name=""):
        self.dim, self.n = int(dim), int(n)
        self.m = self.n ** self.dim
        self.rowptr, self.col, self.val = rowptr, col, val
        self.r_diag = np.asarray(r_diag, np.float64)
        self.p = len(rowptr) - 1
        self.kparams = dict(theta=theta, ell=ell, gamma=gamma)
        self.n_c, self.precision, self.prior, self.sparse = n_c, precision, prior, sparse
        self.psd_guard = psd_guard
        self.name = name

    def options(self, tune_cache=None):
        return F.make_options(self.n_c, self.precision, False, graph=True, sparse=self.sparse,
                              tune_cache=tune_cache, psd_guard=self.psd_guard)

    def plan(self, tune_cache=None):
        pr, keep = F.problem_from_csr(self.dim, self.n, self.rowptr, self.col, self.val,
                                      self.r_diag, prior=self.prior, device="cpu",
                                      **self.kparams)
        return F.plan(pr, self.options(tune_cache))


class _Stream:
    def __init__(self, spec, resident_bytes, scratch_bytes):
        self.spec = spec
        # the resident region plus the stream's output buffers (x_hat, diag P)
        self.resident_bytes = int(resident_bytes) + 16 * spec.m
        self.scratch_bytes = int(scratch_bytes)
        self.filter = None          # HikfFilter while admitted
        self.saved = None           # host copies of (x, var, C) while evicted
        self.queue = collections.deque()     # requests waiting to be issued
        self.inflight = collections.deque()  # (request, event) issued, not yet seen done
        self.slot = None
        self.last_use = 0.0
        self.steps_done = 0
        self.x_out = None
        self.v_out = None


class Request:
    __slots__ = ("rid", "stream", "arrival", "y", "issued", "done", "record")

    def __init__(self, rid, stream, arrival, y, record=False):
        self.rid, self.stream, self.arrival, self.y = rid, stream, arrival, y
        self.issued = self.done = None
        self.record = record        # keep this request's x_hat / diag P on the host


class Server:
    """The serving loop.  specs: StreamSpec per stream; budget_bytes: HBM
    the filters' resident regions may use together; slots: device streams
    on which steps of different filters overlap."""

    def __init__(self, specs, budget_bytes, slots=8, tune_cache=None):
        self.tune_cache = tune_cache
        self.budget = int(budget_bytes)
        self.streams = []
        for s in specs:
            info = s.plan(tune_cache)
            if info.resident_bytes > self.budget:
                raise ValueError(f"stream {s.name}: resident region {info.resident_bytes} B "
                                 f"exceeds the whole budget {self.budget} B")
            self.streams.append(_Stream(s, info.resident_bytes, info.scratch_bytes))
        self.dev_streams = [torch.cuda.Stream() for _ in range(slots)]
        self.free_slots = list(range(slots))
        self.used = 0
        self.stats = collections.Counter()
        self.outputs = {}           # rid -> (x, var) for recorded requests

    # ---------------------------------------------------------------- memory
    def _evict_for(self, need):
        """Evict idle admitted streams, least recently used first, until
        `need` more bytes fit; False if that is impossible now."""
        idle = sorted((st for st in self.streams
                       if st.filter is not None and not st.queue and not st.inflight),
                      key=lambda st: st.last_use)
        for st in idle:
            if self.used + need <= self.budget:
                break
            self._evict(st)
        return self.used + need <= self.budget

    def _evict(self, st):
        x, v, c, ps, info = st.filter.export_checkpoint()
        # pinned host copies (torch caches the pinned blocks, so the next
        # eviction of a similar stream reuses them): the transfers run at
        # full PCIe rate in both directions
        saved = []
        for t in (x, v, c, ps):
            h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
            h.copy_(t, non_blocking=True)
            saved.append(h)
        torch.cuda.current_stream().synchronize()
        st.saved = (*saved, info)
        st.filter.close()
        st.filter = None
        st.x_out = st.v_out = None
        self.used -= st.resident_bytes
        self.stats["evictions"] += 1

    def _admit(self, st, dev_stream):
        """Build the stream's filter on dev_stream (its FMM runs there)."""
        s = st.spec
        pr, keep = F.problem_from_csr(s.dim, s.n, s.rowptr, s.col, s.val, s.r_diag,
                                      prior=s.prior, **s.kparams)
        with torch.cuda.stream(dev_stream):
            f = F.HikfFilter(pr, s.options(self.tune_cache), keep, stream=dev_stream)
            if st.saved is not None:
                x, v, c, ps = (t.to("cuda", non_blocking=True) for t in st.saved[:4])
                f.import_checkpoint(x, v, c, ps, st.saved[4], stream=dev_stream)
                st.saved = None
                self.stats["readmissions"] += 1
            st.x_out = torch.empty(s.m, dtype=torch.float64, device="cuda")
            st.v_out = torch.empty(s.m, dtype=torch.float64, device="cuda")
        st.filter = f
        self.used += st.resident_bytes
        self.stats["admissions"] += 1

    # ---------------------------------------------------------------- loop
    def _issue(self, st):
        ds = self.dev_streams[st.slot]
        while st.queue:
            rq = st.queue.popleft()
            st.filter.step(rq.y, st.x_out, st.v_out, stream=ds)
            if rq.record:
                with torch.cuda.stream(ds):
                    self.outputs[rq.rid] = (st.x_out.to("cpu", non_blocking=False),
                                            st.v_out.to("cpu", non_blocking=False))
            ev = torch.cuda.Event()
            ev.record(ds)
            rq.issued = time.perf_counter()
            st.inflight.append((rq, ev))
            self.stats["issued"] += 1

    def _retire(self, now):
        done = []
        for st in self.streams:
            while st.inflight and st.inflight[0][1].query():
                rq, _ = st.inflight.popleft()
                rq.done = now
                st.steps_done += 1
                st.last_use = now
                done.append(rq)
            if st.slot is not None and not st.inflight and not st.queue:
                self.free_slots.append(st.slot)
                st.slot = None
        return done

    def run(self, requests):
        """Serve `requests` (sorted by arrival; arrival in seconds from the
        start).  Returns the completed requests."""
        t0 = time.perf_counter()
        i, n = 0, len(requests)
        finished = []
        order = collections.deque()          # streams with queued work, FIFO by head arrival
        while len(finished) < n:
            now = time.perf_counter() - t0
            while i < n and requests[i].arrival <= now:
                st = self.streams[requests[i].stream]
                if not st.queue and st not in order:
                    order.append(st)
                st.queue.append(requests[i])
                i += 1
            finished.extend(self._retire(now))
            progressed = False
            for _ in range(len(order)):
                st = order.popleft()
                if not st.queue:
                    continue
                if st.slot is None:
                    if not self.free_slots:
                        order.append(st)
                        continue
                    if st.filter is None:
                        if not self._evict_for(st.resident_bytes):
                            order.append(st)         # wait for memory to free up
                            continue
                        slot = self.free_slots.pop()
                        st.slot = slot
                        self._admit(st, self.dev_streams[slot])
                    else:
                        st.slot = self.free_slots.pop()
                self._issue(st)
                progressed = True
            if not progressed:
                nxt = requests[i].arrival - (time.perf_counter() - t0) if i < n else 0.0
                if nxt > 0:
                    time.sleep(min(nxt, 2e-4))
        torch.cuda.synchronize()
        return finished

    def final_states(self):
        """(x_hat, diag P) of every stream, from its filter or its saved copy."""
        out = []
        for st in self.streams:
            if st.filter is not None:
                x, v, _ = st.filter.export_state()
                out.append((x.cpu(), v.cpu()))
            elif st.saved is not None:
                out.append((st.saved[0], st.saved[1]))
            else:
                out.append(None)
        torch.cuda.synchronize()
        return out

    def query(self):
        return [st.filter.query() if st.filter is not None else None for st in self.streams]

    def close(self):
        for st in self.streams:
            if st.filter is not None:
                st.filter.close()
                st.filter = None


def run_sequential(specs, requests, tune_cache=None, filters=None):
    """The plain path: one filter at a time, each request stepped and waited
    for before the next is looked at (arrival order, real time).  Returns
    the filters (pass them back in to continue them)."""
    if filters is None:
        filters = [None] * len(specs)
    outs = {}
    t0 = time.perf_counter()
    for rq in requests:
        now = time.perf_counter() - t0
        if rq.arrival > now:
            time.sleep(rq.arrival - now)
        k = rq.stream
        if filters[k] is None:
            s = specs[k]
            pr, keep = F.problem_from_csr(s.dim, s.n, s.rowptr, s.col, s.val, s.r_diag,
                                          prior=s.prior, **s.kparams)
            filters[k] = F.HikfFilter(pr, s.options(tune_cache), keep)
        if k not in outs:
            m = specs[k].m
            outs[k] = (torch.empty(m, dtype=torch.float64, device="cuda"),
                       torch.empty(m, dtype=torch.float64, device="cuda"))
        rq.issued = time.perf_counter()
        filters[k].step(rq.y, outs[k][0], outs[k][1])
        torch.cuda.current_stream().synchronize()
        rq.done = time.perf_counter() - t0
    return filters


def latency_summary(requests, wall):
    lat = np.array([(rq.done - rq.arrival) for rq in requests]) * 1e3
    return {"requests": len(requests), "wall_s": round(wall, 3),
            "achieved_per_s": round(len(requests) / wall, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(np.mean(lat)), 3)}
