"""Served form of the query path: several resident models, requests batched
into shared launches.

A request is (model, host query points).  Requests reach the scheduling loop
in one of two ways: ``run`` replays a list of requests with given arrival
times (benchmarks, tests), and ``submit`` hands one request from a live
producer to a loop running on its own thread and returns a
``concurrent.futures.Future`` of its (w, inside).  Either way the loop

* splits each admitted request into pieces of at most ``chunk`` queries, so a
  large request cannot hold back small ones behind it;
* keeps ``n_slots`` launches in flight, one per HIP stream (default 4,
  HIP's default number of hardware queues per process), so the host-device
  copies of one launch overlap the kernels of others and the tail of one
  launch overlaps the next (measured: 2 slots reached about half the
  saturation throughput of 4 on the 2D serving models);
* fills a free slot with pending pieces in arrival order -- all of one
  dimension (2D and 3D models cannot share a launch), at most
  ``max_launch`` queries -- whose device bytes fit in what is left of the
  byte budget: points and outputs, plus the launch's scratch, charged by an
  upper bound the library's own per-launch figure
  (``gwn_query_scratch_bytes``) never exceeds;
* issues, on the slot's stream: a pinned host -> device copy of the points,
  one ``gwn_query_batch`` over the pieces (the pieces of each model side by
  side as one segment, so the sort interleaves their queries; each piece
  contiguous in the output), and the device -> host copies of the values
  and containment flags; then records an event;
* polls the events, hands the values back to their requests and releases
  their bytes.  A request is complete when its last piece is.

Every query's value depends only on its own point and model: the server
runs its models with per-query far tests (``wave_accept`` = 0, whatever the
parameters given), each lane sums its own terms in the left-first order of
its own traversal, so a request's results equal those of a solo
``gwn_query`` bitwise, whatever it was batched with or cut into (tested).

Latency of a request = completion time (when the loop sees its last event)
minus its arrival time (the time it was offered to the loop).
"""
from __future__ import annotations

import ctypes
import queue
import threading
import time
from collections import deque
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from . import gwn as G


@dataclass
class Request:
    model: int                        # index returned by Server.add_model
    points: np.ndarray                # float64 [n, dim], host
    arrival: float = 0.0              # seconds after the run starts
    rid: int = -1
    w: np.ndarray | None = None       # float64 [n] after completion
    inside: np.ndarray | None = None  # uint8 [n]
    done: float = float("nan")        # completion time, seconds after start
    pieces_left: int = 0
    views: tuple = ()                 # torch views of points, w, inside (host copies)
    future: Future | None = None      # set by Server.submit

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Piece:
    req: Request
    begin: int
    end: int


@dataclass
class _Slot:
    stream: object
    event: object
    pins: dict = field(default_factory=dict)
    busy: bool = False
    pieces: list = field(default_factory=list)
    offsets: list = field(default_factory=list)
    bytes: int = 0
    out_w: object = None
    out_in: object = None
    keep: tuple = ()                  # device buffers held until the event completes
    t_events: tuple = ()              # (start, end) timing events of the launch


class Server:
    """Scheduling loop over resident models (see module docstring)."""

    def __init__(self, budget_bytes: int = 4 << 30, n_slots: int = 4, chunk: int = 1 << 18,
                 max_launch: int = 1 << 20, device: int = 0, record_timing: bool = False):
        import torch
        self.torch = torch
        if n_slots < 1 or chunk < 1 or max_launch < 1 or budget_bytes <= 0:
            raise ValueError("bad server configuration")
        self.device = torch.device("cuda", device)
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.max_launch = int(max_launch)
        self.models: list[G.Model] = []
        self.dims: list[int] = []
        self._scratch_fit: dict = {}          # dim -> (c0, per query)
        with torch.cuda.device(self.device):
            self.slots = [_Slot(torch.cuda.Stream(device=self.device), torch.cuda.Event()) for _ in range(n_slots)]
        self.launches = 0
        self.overflow_reports = 0             # launches that reported an earlier launch's NaN queries
        self.in_flight_bytes = 0
        self.peak_bytes = 0
        self.record_timing = record_timing
        self.timeline: list = []              # (slot, start event, end event) per launch when recording
        self._t_ref = None
        # live producer interface
        self._inbox: queue.Queue = queue.Queue()
        self._thread: threading.Thread | None = None
        self._stop = threading.Event()
        self._loop_error: BaseException | None = None
        self._lock = threading.Lock()

    # -- models ---------------------------------------------------------
    def add_model(self, geometry, params: G.gwn_params | None = None) -> int:
        if self._thread is not None:
            raise RuntimeError("add models before the first submit()")
        # per-query far tests: a request's values then do not depend on how
        # it is cut into pieces or on what shares its launch
        if params is not None:
            p = G.gwn_params()
            ctypes.memmove(ctypes.byref(p), ctypes.byref(params), ctypes.sizeof(p))
            p.wave_accept = 0
            params = p
        m = G.Model(geometry, params)
        self.models.append(m)
        self.dims.append(m.dim)
        if m.dim not in self._scratch_fit:
            self._scratch_fit[m.dim] = self._fit_scratch(m)
        return len(self.models) - 1

    def _fit_scratch(self, m: G.Model):
        """(c0, pq) with c0 + pq n >= the library's scratch bytes of a launch
        of n queries in up to 32 segments, for every n up to max_launch:
        through the library's exact figures at n = 1 and at 2^k - 1, 2^k,
        2^k + 1 (the sizes where its wave spreading and sort passes change),
        with a 2 % and 64 KiB margin for the sizes in between."""
        ns = {1, self.max_launch}
        k = 1
        while (1 << k) <= 2 * self.max_launch:
            ns |= {(1 << k) - 1, 1 << k, (1 << k) + 1}
            k += 1
        c0 = G.gwn_query_scratch_bytes(m.h, 1, 32)
        pq = 0.0
        for n in sorted(ns):
            pq = max(pq, (G.gwn_query_scratch_bytes(m.h, n, 32) - c0) / n)
        return c0 + (64 << 10), pq * 1.02

    def resident_bytes(self) -> int:
        return sum(int(m.bytes()[0]) for m in self.models)

    def launch_bytes(self, dim: int, n: int) -> int:
        """Device bytes charged for a launch of n queries: points, outputs and
        the bound on its scratch."""
        c0, pq = self._scratch_fit[dim]
        return int(n * (8 * dim + 8 + 1) + c0 + pq * n) + 1

    def _piece_size(self, dim: int) -> int:
        share = self.budget // len(self.slots)
        c0, pq = self._scratch_fit[dim]
        n = int((share - c0 - 1) // (8 * dim + 9 + pq))
        if n < 1:
            raise ValueError(f"budget of {self.budget} bytes over {len(self.slots)} slots cannot hold one "
                             f"{dim}D query ({self.launch_bytes(dim, 1)} bytes per launch)")
        return min(self.chunk, n)

    # -- requests ---------------------------------------------------------
    def _prepare(self, r: Request, k: int):
        torch = self.torch
        if not (0 <= r.model < len(self.models)):
            raise ValueError(f"request {k}: unknown model {r.model}")
        pts = np.ascontiguousarray(r.points, dtype=np.float64)
        if not pts.flags.writeable:
            pts = pts.copy()
        if pts.ndim != 2 or pts.shape[1] != self.dims[r.model]:
            raise ValueError(f"request {k}: points must be [n, {self.dims[r.model]}]")
        r.points = pts
        r.rid = k
        r.w = np.empty(pts.shape[0], np.float64)
        r.inside = np.empty(pts.shape[0], np.uint8)
        r.views = (torch.from_numpy(pts), torch.from_numpy(r.w), torch.from_numpy(r.inside))
        r.done = float("nan")

    def _admit(self, r: Request, now: float, pending: deque) -> int:
        """Split an arrived request into pieces; 1 if it completes at once."""
        n = r.points.shape[0]
        if n == 0:
            self._complete(r, now)
            return 1
        step = self._piece_size(self.dims[r.model])
        r.pieces_left = (n + step - 1) // step
        for b in range(0, n, step):
            pending.append(_Piece(r, b, min(n, b + step)))
        return 0

    @staticmethod
    def _complete(r: Request, now: float):
        r.done = now
        if r.future is not None:
            r.future.set_result((r.w, r.inside))

    def _tick(self, pending: deque, now_fn) -> tuple:
        """Retire finished launches and fill free slots: (requests finished,
        launched anything)."""
        finished = 0
        for s in self.slots:
            if s.busy and s.event.query():
                finished += self._retire(s, now_fn())
        launched = False
        for s in self.slots:
            if not s.busy and pending:
                launched |= self._launch(s, pending)
        return finished, launched

    # -- replayed requests --------------------------------------------------
    def run(self, requests: list[Request], closed_loop: bool = False, progress=None) -> dict:
        """Serve ``requests`` to completion.  Arrival times are honoured
        (open loop) unless ``closed_loop``, where all are offered at t = 0.
        ``progress``: optional callable, given a status string about every
        5 s.  Returns throughput and latency statistics."""
        if self._thread is not None:
            raise RuntimeError("run() cannot be used while the submit() loop is active")
        for k, r in enumerate(requests):
            self._prepare(r, k)
            if closed_loop:
                r.arrival = 0.0
        order = sorted(requests, key=lambda r: r.arrival)
        arrivals = deque(order)
        pending: deque[_Piece] = deque()
        n_done = 0
        total_q = sum(r.points.shape[0] for r in requests)
        self.timeline = []
        self._start_clock()
        t0 = time.perf_counter()
        now_fn = lambda: time.perf_counter() - t0
        next_report = 5.0
        while n_done < len(requests):
            now = now_fn()
            if progress is not None and now >= next_report:
                next_report += 5.0
                progress(f"t={now:.1f}s done {n_done}/{len(requests)} pending pieces {len(pending)} "
                         f"launches {self.launches} in flight {self.in_flight_bytes} B")
            while arrivals and arrivals[0].arrival <= now:
                n_done += self._admit(arrivals.popleft(), now, pending)
            finished, launched = self._tick(pending, now_fn)
            n_done += finished
            if not launched and not any(s.busy for s in self.slots) and not pending and arrivals:
                wait = arrivals[0].arrival - now_fn()
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
            elif not launched:
                time.sleep(2e-5)
        wall = now_fn()
        lat = np.array([r.latency for r in requests if r.points.shape[0] > 0])
        return {
            "requests": len(requests), "queries": int(total_q), "wall_s": wall,
            "queries_per_s": total_q / wall if wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else 0.0,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else 0.0,
            "mean_ms": float(lat.mean() * 1e3) if lat.size else 0.0,
            "launches": self.launches, "peak_in_flight_bytes": self.peak_bytes, "budget_bytes": self.budget,
            "overflow_reports": self.overflow_reports,
        }

    # -- live producers ---------------------------------------------------------
    def submit(self, model: int, points) -> Future:
        """Offer one request from a live producer (any thread).  Returns a
        Future of (w float64 [n], inside uint8 [n]); the request is admitted
        by the loop thread, started on the first call, as slots and budget
        free up.  Invalid requests fail their future with ValueError."""
        fut: Future = Future()
        if self._loop_error is not None:
            raise RuntimeError("the serving loop stopped") from self._loop_error
        with self._lock:
            if self._stop.is_set():
                raise RuntimeError("server is closed")
            if self._thread is None:
                self._start_clock()
                self._t0 = time.perf_counter()
                self._thread = threading.Thread(target=self._loop, name="gwn-serve", daemon=True)
                self._thread.start()
        self._inbox.put((model, points, fut, time.perf_counter()))
        return fut

    def _loop(self):
        torch = self.torch
        pending: deque[_Piece] = deque()
        now_fn = lambda: time.perf_counter() - self._t0
        k = 0
        try:
            with torch.cuda.device(self.device):
                while True:
                    idle = not pending and not any(s.busy for s in self.slots)
                    if idle and self._stop.is_set() and self._inbox.empty():
                        return
                    try:
                        item = self._inbox.get(timeout=1e-3) if idle else self._inbox.get_nowait()
                    except queue.Empty:
                        item = None
                    while item is not None:
                        model, pts, fut, t_arr = item
                        r = Request(model, pts, arrival=t_arr - self._t0, future=fut)
                        try:
                            self._prepare(r, k)
                            k += 1
                            self._admit(r, now_fn(), pending)
                        except ValueError as e:
                            fut.set_exception(e)
                        try:
                            item = self._inbox.get_nowait()
                        except queue.Empty:
                            item = None
                    _, launched = self._tick(pending, now_fn)
                    if not launched and not idle:
                        time.sleep(2e-5)
        except BaseException as e:   # hand the failure to every waiting producer
            self._loop_error = e
            for s in self.slots:
                for p in s.pieces:
                    if p.req.future is not None and not p.req.future.done():
                        p.req.future.set_exception(e)
            for p in pending:
                if p.req.future is not None and not p.req.future.done():
                    p.req.future.set_exception(e)
            raise

    # -- launches ---------------------------------------------------------
    def _start_clock(self):
        if self.record_timing:
            with self.torch.cuda.device(self.device):
                self._t_ref = self.torch.cuda.Event(enable_timing=True)
                self._t_ref.record()

    def _pinned(self, s: _Slot, key: str, n: int, dtype):
        torch = self.torch
        buf = s.pins.get(key)
        if buf is None or buf.numel() < n:
            buf = torch.empty(max(n, 1 << 12), dtype=dtype, pin_memory=True)
            s.pins[key] = buf
        return buf[:n]

    def _launch(self, s: _Slot, pending: deque) -> bool:
        torch = self.torch
        dim = self.dims[pending[0].req.model]
        free = self.budget - self.in_flight_bytes
        take, nq = [], 0
        while pending and len(take) < 4096:
            p = pending[0]
            m = p.req.model
            if self.dims[m] != dim:
                break
            cnt = p.end - p.begin
            b = self.launch_bytes(dim, nq + cnt)
            if take and (nq + cnt > self.max_launch or b > free):
                break
            if not take and b > free:
                return False        # wait for bytes to come back
            take.append(pending.popleft())
            nq += cnt
        if not take:
            return False
        nbytes = self.launch_bytes(dim, nq)
        # gather points into the slot's pinned buffer, the pieces of each
        # model next to each other: one segment per model, so the library's
        # space-filling-curve sort interleaves the queries of all requests
        # for that model (denser waves; values do not depend on wave mates)
        take.sort(key=lambda p: p.req.model)
        # (host copies through torch, which splits large ones over threads)
        h_pts = self._pinned(s, "pts", nq * dim, torch.float64)
        hp = h_pts.view(nq, dim)
        offsets = [0]
        seg_models, seg_off = [], [0]
        for p in take:
            c = p.end - p.begin
            hp[offsets[-1]:offsets[-1] + c].copy_(p.req.views[0][p.begin:p.end])
            offsets.append(offsets[-1] + c)
            if seg_models and seg_models[-1] == p.req.model:
                seg_off[-1] = offsets[-1]
            else:
                seg_models.append(p.req.model)
                seg_off.append(offsets[-1])
        with torch.cuda.stream(s.stream):
            t_start = None
            if self.record_timing:
                t_start = torch.cuda.Event(enable_timing=True)
                t_start.record(s.stream)
            d_pts = torch.empty((nq, dim), dtype=torch.float64, device=self.device)
            d_w = torch.empty(nq, dtype=torch.float64, device=self.device)
            d_in = torch.empty(nq, dtype=torch.uint8, device=self.device)
            d_pts.view(-1).copy_(h_pts, non_blocking=True)
            handles = [self.models[m].h for m in seg_models]
            # A query that hit a traversal or near-field limit comes back NaN
            # in its own request; the library reports the count on the next
            # call on that model, which then launches nothing.  Such a report
            # belongs to an earlier launch: count it and launch again (at most
            # one report per model of the batch).
            for attempt in range(len(handles) + 1):
                try:
                    G.gwn_query_batch(handles, np.asarray(seg_off, np.int64), d_pts, d_w, d_in, s.stream)
                    break
                except G.GwnError as e:
                    if e.status != G.GWN_EOVERFLOW or attempt == len(handles):
                        raise
                    self.overflow_reports += 1
            h_w = self._pinned(s, "w", nq, torch.float64)
            h_in = self._pinned(s, "in", nq, torch.uint8)
            h_w.copy_(d_w, non_blocking=True)
            h_in.copy_(d_in, non_blocking=True)
            if self.record_timing:
                t_end = torch.cuda.Event(enable_timing=True)
                t_end.record(s.stream)
                self.timeline.append((self.slots.index(s), t_start, t_end))
            s.event.record(s.stream)
        s.busy = True
        s.pieces = take
        s.offsets = offsets
        s.bytes = nbytes
        s.out_w, s.out_in = h_w, h_in
        s.keep = (d_pts, d_w, d_in)
        self.in_flight_bytes += nbytes
        self.peak_bytes = max(self.peak_bytes, self.in_flight_bytes)
        self.launches += 1
        return True

    def _retire(self, s: _Slot, now: float) -> int:
        w, ins = s.out_w, s.out_in
        finished = 0
        for k, p in enumerate(s.pieces):
            a, b = s.offsets[k], s.offsets[k + 1]
            p.req.views[1][p.begin:p.end].copy_(w[a:b])
            p.req.views[2][p.begin:p.end].copy_(ins[a:b])
            p.req.pieces_left -= 1
            if p.req.pieces_left == 0:
                self._complete(p.req, now)
                finished += 1
        self.in_flight_bytes -= s.bytes
        s.busy = False
        s.pieces, s.offsets, s.keep = [], [], ()
        s.bytes = 0
        return finished

    def launch_intervals(self) -> list:
        """With record_timing: (slot, start ms, end ms) of every launch of the
        last run, from HIP events on the slot streams, relative to the run's
        start (call after the run has finished)."""
        self.torch.cuda.synchronize(self.device)
        return [(k, self._t_ref.elapsed_time(a), self._t_ref.elapsed_time(b)) for k, a, b in self.timeline]

    def close(self):
        """Finish the submitted work, stop the loop thread, free the models."""
        with self._lock:
            self._stop.set()
        if self._thread is not None:
            self._thread.join()
        for m in self.models:
            m.close()
        self.models = []


def poisson_requests(rng, n_requests: int, rate: float, models: list[int], sizes: np.ndarray, points_fn):
    """Requests with exponential inter-arrival times of mean 1/rate seconds;
    model k = models[i], size sizes[i], points from points_fn(model, n, i)."""
    gaps = -np.log(1.0 - rng.uniform(n_requests, 0.0, 1.0)) / rate
    t = np.cumsum(gaps)
    return [Request(models[i], points_fn(models[i], int(sizes[i]), i), float(t[i])) for i in range(n_requests)]
