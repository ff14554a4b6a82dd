"""Serving loop for alignment-plot jobs: admission by HBM footprint and
continuous batching.

A job is one plot request (strings x and y, window w, alphabet, bitmap
threshold, optional indel output; optionally step sizes and, instead of the
dense bitmap, the list of dots at or above the threshold, which holds far
fewer bytes than the dense outputs of a large plot).  The server keeps a FIFO of waiting jobs
and admits the head while its device footprint (resident letter codes plus
its outputs) fits the memory budget and a job slot is free.  Admitted jobs
are launched together as one batch (persistent work-stealing launches,
``wlcs_batch``) on one of several streams, so jobs that arrive while earlier
batches run start on a free stream and overlap them on the device.  A batch
is enqueued as sub-batches of increasing job cost, each with its own
completion event, so a cheap job completes without waiting for the costly
ones launched beside it; a job's completion frees its footprint and slot,
which admits more jobs.  Latency is measured from a job's arrival to the
completion of its sub-batch on the device.

The scheduler only talks to an executor: ``GpuExecutor`` drives the library on
one GPU; the tests use a fake executor with a virtual clock to check
admission, ordering and continuous admission without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from dataclasses import dataclass, field

import numpy as np

# Padding the library allocates per resident pair (letter codes, in bytes):
# x gets 384 extra 16-bit codes and y two maximal tiles plus a window.
PAIR_PAD_BYTES = 2 * (384 + 2 * 32768 + 448)


@dataclass
class Request:
    jid: int
    x: np.ndarray
    y: np.ndarray
    w: int
    alphabet: bytes
    threshold: int | None = None
    indel: bool = True
    want_plot: bool = False
    arrival: float = 0.0       # seconds on the server's clock
    hx: int = 1                # step sizes (Section 3): x-windows r*hx, y-windows c*hy
    hy: int = 1
    dot_cap: int | None = None  # list the dots (up to dot_cap records) instead of a bitmap


@dataclass
class JobState:
    req: Request
    admitted: float = -1.0
    launched: float = -1.0
    done: float = -1.0
    footprint: int = 0
    results: dict | None = None
    batch_id: int = -1
    retries: int = 0           # reruns with a longer dot list
    # "pending" until the job ends: "done", "rejected" (can never fit),
    # "failed" (its launch failed; error holds why), "cancelled", "timed_out"
    status: str = "pending"
    error: str | None = None
    cancel_requested: bool = False  # cancelled while its work was on the device
    timed_out: bool = False         # its batch outran the server's batch timeout


class LaunchError(RuntimeError):
    """A batch was launched in part: `unlaunched` are the jobs that were not
    (the executor keeps track of the rest), `cause` the original error."""

    def __init__(self, unlaunched: list, cause: BaseException):
        super().__init__(f"{len(unlaunched)} jobs not launched: {cause!r}")
        self.unlaunched, self.cause = unlaunched, cause


def is_out_of_memory(e: BaseException) -> bool:
    """Whether a launch failed for lack of device memory (the library's
    WLCS_ENOMEM, or the allocator's out-of-memory error)."""
    e = getattr(e, "cause", e)
    if getattr(e, "status", None) == -5:
        return True
    return type(e).__name__ in ("OutOfMemoryError", "MemoryError") or "out of memory" in str(e).lower()


def windows(length: int, w: int) -> int:
    return max(length - w, 0)


DOT_BYTES = 12  # one wlcs_dot record


def footprint_bytes(req: Request) -> int:
    """HBM a job holds while admitted: its resident codes and its outputs."""
    rows = -(-windows(req.x.size, req.w) // req.hx)
    cols = -(-windows(req.y.size, req.w) // req.hy)
    b = 2 * (req.x.size + req.y.size) + PAIR_PAD_BYTES
    if req.want_plot:
        b += rows * cols
    if req.threshold is not None and req.dot_cap is None and req.hy == 1:
        b += rows * ((cols + 63) // 64) * 8
    if req.dot_cap is not None:
        b += DOT_BYTES * req.dot_cap + 8
    if req.indel:
        b += rows * cols * 2
    return b


# A batch is enqueued as sub-batches of increasing cost with an event each; a
# job up to this many times the cost of the cheapest job of the current
# sub-batch joins it, a costlier one starts the next.  Every sub-batch costs
# its own launches and tail, so too fine a split lowers capacity (measured on
# the serving workload: 16 keeps 98.5% of the capacity of one event per
# batch and lowers p99 by 10-20% at 0.5-0.75 of capacity; 2 loses 20%).
SUB_BATCH_RATIO = 16.0


def job_cost(js) -> float:
    """Combing work of a job: x-windows x y-windows x w (its cells, up to the
    steps' and the window's constant factors)."""
    r = js.req
    return float(max(r.x.size - r.w, 1)) / r.hx * max(r.y.size - r.w, 1) * r.w


# Batch tiles that favour latency: short tiles give every job many units, so a
# job spreads over the device even when few others run beside it.
LATENCY_TILES = {(1, 64): 512, (65, 128): 1024}
LATENCY_GRID = 16
# A job with fewer units than this under those tiles gets shorter ones
# (wlcs_ctx_set_batch_min_units): a small job then spreads over about one
# unit per SIMD of the device instead of combing its tiles on a few waves.
LATENCY_MIN_UNITS = 1024


# The serving loop's waits.  While batches run it polls their events without
# sleeping (POLL_SLEEP_S 0).  With nothing running it sleeps until the next
# arrival, waking ARRIVAL_EARLY_S early and polling the clock from there,
# since a sleep overshoots by tens of microseconds.
POLL_SLEEP_S = 0.0
ARRIVAL_EARLY_S = 200e-6


# Streams of the executors, per device, shared by every executor of the
# process: torch's caching allocator keeps freed blocks per stream, so
# executors on new streams could not reuse the output memory their
# predecessors cached and would map fresh device memory each time (until the
# device is full and the allocator has to release everything at once).
_STREAM_POOL: dict = {}


def _streams(torch, dev, count: int) -> list:
    pool = _STREAM_POOL.setdefault(dev.index, [])
    while len(pool) < count:
        pool.append(torch.cuda.Stream(device=dev))
    return pool[:count]


class GpuExecutor:
    """Runs batches on one GPU through libwlcs, one stream per concurrent batch
    (from the process's shared stream pool), each batch as sub-batches with
    their own completion events.  Without a context of its own it makes one
    with the latency tiles (and shorter ones for jobs too small to fill the
    device, LATENCY_MIN_UNITS).  With d2h_bitmaps each job's bitmap is also copied
    to pinned host memory on the stream before its sub-batch's completion event
    (result "bitmap_host"), so that a job's latency runs until its result is on
    the host."""

    def __init__(self, device: int = 0, streams: int = 4, ctx=None, d2h_bitmaps: bool = False):
        import torch

        import paper_0909_2000_amd as wl
        self.torch, self.wl = torch, wl
        self.dev = torch.device("cuda", device)
        if ctx is None:
            ctx = wl.Context(device)
            for (lo, hi), t in LATENCY_TILES.items():
                ctx.set_batch_tile(lo, hi, t)
            ctx.set_batch_grid(LATENCY_GRID)
            ctx.set_batch_min_units(LATENCY_MIN_UNITS)
        self.ctx = ctx
        self.d2h = d2h_bitmaps
        self.streams = _streams(torch, self.dev, streams)
        self.busy = [None] * streams  # per stream: (event, batch_id) or None
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def free_stream(self):
        for k, b in enumerate(self.busy):
            if b is None:
                return k
        return None

    def launch(self, batch_id: int, jobs: list) -> None:
        """Enqueue the jobs on a free stream as sub-batches of increasing cost
        (a job more than SUB_BATCH_RATIO times the cheapest of the current
        sub-batch starts the next), each followed by its own completion event:
        the batch's GPU work is the same, but cheap jobs complete without
        waiting for the expensive ones launched beside them."""
        k = self.free_stream()
        s = self.streams[k]
        subs = []
        for js in sorted(jobs, key=job_cost):
            if subs and job_cost(js) <= SUB_BATCH_RATIO * job_cost(subs[-1][0]):
                subs[-1].append(js)
            else:
                subs.append([js])
        pending = []
        try:
            for sub in subs:
                pending.append((self._launch_sub(s, sub), sub))
        except Exception as e:  # e.g. no device memory left for a sub-batch's pair or outputs
            launched = [js for _, sub in pending for js in sub]
            if pending:
                self.busy[k] = (pending, batch_id)  # what was enqueued completes as usual
            done = {id(js) for js in launched}
            for js in jobs:
                if id(js) not in done:
                    js.results = None
            raise LaunchError([js for js in jobs if id(js) not in done], e) from e
        self.busy[k] = (pending, batch_id)

    def _launch_sub(self, s, jobs: list):
        specs = []
        for js in jobs:
            r = js.req
            pair = self.ctx.pair(r.x, r.y, alphabet=r.alphabet, stream=s)
            sp = {"pair": pair, "w": r.w, "threshold": r.threshold, "indel": r.indel,
                  "want_plot": r.want_plot, "hx": r.hx, "hy": r.hy}
            if r.dot_cap is not None:
                sp["dot_cap"] = r.dot_cap
            specs.append(sp)
        with self.torch.cuda.stream(s):
            results = self.ctx.batch(specs, stream=s)
            if self.d2h:
                for res in results:
                    if "bitmap" in res:
                        host = self.torch.empty(res["bitmap"].shape, dtype=res["bitmap"].dtype, pin_memory=True)
                        host.copy_(res["bitmap"], non_blocking=True)
                        res["bitmap_host"] = host
            ev = self.torch.cuda.Event()
            ev.record(s)
        for js, res, sp in zip(jobs, results, specs):
            js.results = res
            js.results["_pair"] = sp["pair"]  # keeps the resident codes alive until the job is done
        return ev

    def dot_counts(self, jobs: list) -> list:
        """Dots each finished job found (None for jobs without a list), read
        back in one copy."""
        idx = [k for k, js in enumerate(jobs) if js.results and "dot_count" in js.results]
        out = [None] * len(jobs)
        if idx:
            vals = self.torch.cat([jobs[k].results["dot_count"] for k in idx]).cpu().tolist()
            for k, v in zip(idx, vals):
                out[k] = int(v)
        return out

    def poll_jobs(self) -> list:
        """(batch id, jobs finished since the last call, whether the whole
        batch is done) for every batch with newly finished sub-batches; a
        stream is free again once its batch is done."""
        out = []
        for k, b in enumerate(self.busy):
            if b is None:
                continue
            pending, bid = b
            fin = []
            while pending and pending[0][0].query():  # sub-batches finish in stream order
                fin.extend(pending.pop(0)[1])
            if fin or not pending:
                out.append((bid, fin, not pending))
            if not pending:
                self.busy[k] = None
        return out

    def poll(self) -> list:
        """Batch ids whose work has finished on the device (whole batches)."""
        return [bid for bid, _, done in self.poll_jobs() if done]

    def idle_wait(self):
        """Between polls while batches run: with POLL_SLEEP_S 0 the loop keeps
        polling the completion events (one host core busy); a sleep, however
        short, lasts tens of microseconds more than asked (timer slack), which
        every job's latency pays."""
        if POLL_SLEEP_S > 0:
            time.sleep(POLL_SLEEP_S)


class Server:
    def __init__(self, executor, budget_bytes: int, max_jobs: int = 256, max_batch: int = 64,
                 keep_results: bool = True, on_done=None, batch_timeout_s: float | None = None):
        """on_done(request, results), if given, is called once per job when it
        completes (its sub-batch's event has fired), before the results are
        released (keep_results=False) -- e.g. to check or copy them.
        batch_timeout_s: a batch still running this long after its launch (on
        the executor's clock) has its unfinished jobs marked timed out; their
        memory is released only when the device work ends, and their results
        are dropped."""
        self.ex = executor
        self.on_done = on_done
        self.batch_timeout = batch_timeout_s
        self.budget = int(budget_bytes)
        self.max_jobs = max_jobs
        self.max_batch = max_batch
        self.keep = keep_results
        self.waiting: collections.deque = collections.deque()
        self.admitted: list = []           # admitted, not yet launched
        self.running: dict = {}            # batch_id -> list of JobState
        self.jobs: dict = {}
        self.in_use = 0                    # bytes held by admitted or running jobs
        self.active = 0                    # jobs admitted or running
        self.peak_use = 0
        self.next_batch = 0
        self.rejected: list = []
        self.admit_log: list = []          # (time, jid) in admission order
        self.overlaps = 0                  # launches made while another batch ran
        self.retries = 0                   # jobs rerun because their dot list was too short
        self.launch_retries = 0            # jobs put back in the queue after a launch ran out of memory
        self.failed: list = []
        self.cancelled: list = []
        self.timed_out: list = []
        self.launched_at: dict = {}        # batch id -> executor time of its launch

    # -- client side -----------------------------------------------------
    def submit(self, req: Request) -> int:
        js = JobState(req, footprint=footprint_bytes(req))
        self.jobs[req.jid] = js
        if js.footprint > self.budget:
            js.done = self.ex.now()
            js.status = "rejected"
            self.rejected.append(req.jid)  # can never fit
        else:
            self.waiting.append(js)
        return req.jid

    def poll(self, jid: int) -> bool:
        return self.jobs[jid].done >= 0

    def status(self, jid: int) -> str:
        return self.jobs[jid].status

    def cancel(self, jid: int) -> bool:
        """Cancel a job that has not ended: a waiting or admitted job leaves at
        once (its memory is released); a job whose work is on the device keeps
        its memory until that work ends, then its results are dropped.  False
        if the job had already ended."""
        js = self.jobs.get(jid)
        if js is None or js.done >= 0 or js.cancel_requested:
            return False
        now = self.ex.now()
        if js in self.waiting:
            self.waiting.remove(js)
        elif js in self.admitted:
            self.admitted.remove(js)
            self.in_use -= js.footprint
            self.active -= 1
        else:  # running: ends with its sub-batch
            js.cancel_requested = True
            return True
        js.status, js.done, js.results = "cancelled", now, None
        self.cancelled.append(jid)
        return True

    def result(self, jid: int) -> dict | None:
        return self.jobs[jid].results

    # -- scheduler -------------------------------------------------------
    def _reap(self):
        if hasattr(self.ex, "poll_jobs"):  # jobs complete with their own sub-batch
            finished = self.ex.poll_jobs()
        else:  # whole batches
            finished = [(bid, self.running[bid], True) for bid in self.ex.poll()]
        for bid, batch, batch_done in finished:
            now = self.ex.now()
            if batch_done:
                self.running.pop(bid)
                self.launched_at.pop(bid, None)
            else:
                done_ids = {id(js) for js in batch}
                self.running[bid] = [js for js in self.running[bid] if id(js) not in done_ids]
            counts = self.ex.dot_counts(batch) if hasattr(self.ex, "dot_counts") else [None] * len(batch)
            retry = []
            for js, found in zip(batch, counts):
                self.in_use -= js.footprint
                self.active -= 1
                if js.cancel_requested or js.timed_out:
                    js.status = "cancelled" if js.cancel_requested else "timed_out"
                    (self.cancelled if js.cancel_requested else self.timed_out).append(js.req.jid)
                    js.done, js.results = now, None
                    continue
                if found is not None and js.req.dot_cap is not None and found > js.req.dot_cap:
                    # the list was too short: rerun the job with room for every dot
                    js.req = dataclasses.replace(js.req, dot_cap=found)
                    js.footprint = footprint_bytes(js.req)
                    js.results = None
                    js.retries += 1
                    self.retries += 1
                    retry.append(js)
                    continue
                js.done = now
                js.status = "done"
                if self.on_done is not None:
                    self.on_done(js.req, js.results)
                if not self.keep:
                    js.results = None
            for js in reversed(retry):  # ahead of every job that arrived later
                if js.footprint > self.budget:
                    js.done = now
                    js.status = "rejected"
                    self.rejected.append(js.req.jid)
                else:
                    self.waiting.appendleft(js)

    def _admit(self):
        while self.waiting and self.active < self.max_jobs:
            head = self.waiting[0]
            if self.in_use + head.footprint > self.budget:
                break  # FIFO: the head waits for memory, nobody overtakes it
            self.waiting.popleft()
            head.admitted = self.ex.now()
            self.in_use += head.footprint
            self.active += 1
            self.peak_use = max(self.peak_use, self.in_use)
            self.admitted.append(head)
            self.admit_log.append((head.admitted, head.req.jid))

    def _launch(self):
        while self.admitted and self.ex.free_stream() is not None:
            batch, self.admitted = self.admitted[:self.max_batch], self.admitted[self.max_batch:]
            bid = self.next_batch
            self.next_batch += 1
            if self.running:
                self.overlaps += 1
            now = self.ex.now()
            for js in batch:
                js.launched = now
                js.batch_id = bid
            self.running[bid] = batch
            self.launched_at[bid] = now
            try:
                self.ex.launch(bid, batch)
            except Exception as e:
                self._launch_failed(bid, batch, e)

    def _launch_failed(self, bid: int, batch: list, e: Exception):
        """A launch failed for some (LaunchError) or all of the batch's jobs.
        Jobs that were not launched give their memory back; if they failed for
        lack of device memory while other batches hold some, they return to
        the head of the queue (in order) to be admitted again once memory is
        released; otherwise they fail with the error recorded."""
        left = e.unlaunched if isinstance(e, LaunchError) else list(batch)
        ids = {id(js) for js in left}
        rest = [js for js in batch if id(js) not in ids]
        if rest:
            self.running[bid] = rest
        else:
            self.running.pop(bid, None)
            self.launched_at.pop(bid, None)
        for js in left:
            self.in_use -= js.footprint
            self.active -= 1
            js.results, js.batch_id, js.launched = None, -1, -1.0
        now = self.ex.now()
        if is_out_of_memory(e) and self.running:
            for js in reversed(left):
                self.waiting.appendleft(js)
            self.launch_retries += len(left)
        else:
            for js in left:
                js.status, js.error, js.done = "failed", repr(getattr(e, "cause", e)), now
                self.failed.append(js.req.jid)

    def _check_timeouts(self):
        if self.batch_timeout is None:
            return
        now = self.ex.now()
        for bid, batch in self.running.items():
            if now - self.launched_at.get(bid, now) > self.batch_timeout:
                for js in batch:
                    js.timed_out = True

    def step(self):
        self._reap()
        self._check_timeouts()
        self._admit()
        self._launch()

    def busy(self) -> bool:
        return bool(self.waiting or self.admitted or self.running)

    def run(self, requests: list) -> dict:
        """Feed requests at their arrival times (server clock) until all are done."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        k = 0
        while k < len(reqs) or self.busy():
            now = self.ex.now()
            while k < len(reqs) and reqs[k].arrival <= now:
                self.submit(reqs[k])
                k += 1
            self.step()
            if hasattr(self.ex, "advance"):
                nxt = reqs[k].arrival if k < len(reqs) else None
                self.ex.advance(nxt)
            elif k < len(reqs) and not self.busy():
                gap = reqs[k].arrival - self.ex.now() - ARRIVAL_EARLY_S
                if gap > 0:
                    time.sleep(min(gap, 1e-3))
            else:
                self.ex.idle_wait()
        return self.report()

    def report(self) -> dict:
        lat = np.array([js.done - js.req.arrival for js in self.jobs.values() if js.status == "done"])
        first = min((js.req.arrival for js in self.jobs.values()), default=0.0)
        last = max((js.done for js in self.jobs.values()), default=0.0)
        cells = sum(float(js.req.x.size) * js.req.y.size * js.req.w for js in self.jobs.values()
                    if js.status == "done")
        ndone = sum(1 for js in self.jobs.values() if js.status == "done")
        span = max(last - first, 1e-9)
        return {
            "jobs": len(self.jobs), "rejected": len(self.rejected),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None,
            "span_s": span, "jobs_per_s": ndone / span,
            "window_cells_per_s": cells / span, "batches": self.next_batch,
            "overlapped_launches": self.overlaps, "peak_bytes": self.peak_use,
            "budget_bytes": self.budget, "dot_list_reruns": self.retries,
            "failed": len(self.failed), "cancelled": len(self.cancelled), "timed_out": len(self.timed_out),
            "launch_retries": self.launch_retries,
        }


def default_dot_cap(rows: int, cols: int) -> int:
    """First list capacity of a sparse job: one record per 64 window pairs
    (about 1.5 times the bytes of the job's bitmap), at least 4096.  A job
    with more dots is rerun with an exact list (Server._reap)."""
    return max(4096, rows * cols // 64)


def requests_from_workload(jobs, rate_scale: float = 1.0, want_plot: bool = False, dots: bool = False,
                           hx: int = 1, hy: int = 1) -> list:
    """Turn workloads.serving_jobs() into Requests; arrival times are divided
    by rate_scale (so rate_scale > 1 compresses the stream).  dots: ask for
    the dot list (with its indel distances) instead of the dense bitmap and
    indel matrices."""
    out = []
    for j in jobs:
        p = j.pair
        cap = None
        if dots:
            cap = default_dot_cap(-(-windows(p.x.size, p.w) // hx), -(-windows(p.y.size, p.w) // hy))
        out.append(Request(j.jid, p.x, p.y, p.w, p.alphabet, threshold=j.threshold, indel=not dots,
                           want_plot=want_plot, arrival=j.arrival / rate_scale, hx=hx, hy=hy, dot_cap=cap))
    return out
