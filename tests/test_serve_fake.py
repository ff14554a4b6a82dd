"""Serving scheduler on the CPU, with a fake executor on a virtual clock.

The fake executor runs each batch for a time proportional to its window-cells
and computes every job's outputs with the oracle, so these tests check the
scheduler itself: the memory budget is never exceeded, admission is FIFO,
jobs are admitted and launched while earlier batches still run, a job's
result in the mix equals the job computed alone, and impossible jobs are
rejected.
"""
import numpy as np
import pytest

import workloads
from paper_0909_2000_amd import serve


class FakeExecutor:
    def __init__(self, oracle, streams=2, rate=2e6, overhead=1e-3):
        self.oracle = oracle
        self.t = 0.0
        self.busy = [None] * streams
        self.rate, self.overhead = rate, overhead
        self.launch_log = []  # (time, batch_id, running batch ids at launch)

    def now(self):
        return self.t

    def free_stream(self):
        for k, b in enumerate(self.busy):
            if b is None:
                return k
        return None

    def launch(self, batch_id, jobs):
        k = self.free_stream()
        assert k is not None
        running = [b[1] for b in self.busy if b is not None]
        cells = sum(float(j.req.x.size) * j.req.y.size * j.req.w for j in jobs)
        self.busy[k] = (self.t + self.overhead + cells / self.rate, batch_id)
        self.launch_log.append((self.t, batch_id, running))
        for j in jobs:
            r = j.req
            plot = self.oracle.wlcs_strided(r.x, r.y, r.w, r.hx, r.hy)
            res = {}
            if r.want_plot:
                res["wlcs"] = plot
            if r.threshold is not None and r.dot_cap is None and r.hy == 1:
                res["bitmap"] = self.oracle.dot_bitmap(plot, r.threshold)
            if r.dot_cap is not None:
                full = self.oracle.dot_list(plot, r.w, r.threshold, r.hx, r.hy)
                res["dots"], res["dot_count"] = full[:r.dot_cap], full.size
            if r.indel:
                res["indel"] = self.oracle.indel(plot, r.w)
            j.results = res

    def dot_counts(self, jobs):
        return [js.results.get("dot_count") if js.results else None for js in jobs]

    def poll(self):
        done = []
        for k, b in enumerate(self.busy):
            if b is not None and b[0] <= self.t + 1e-12:
                done.append(b[1])
                self.busy[k] = None
        return done

    def advance(self, next_arrival):
        fins = [b[0] for b in self.busy if b is not None]
        cands = fins + ([next_arrival] if next_arrival is not None else [])
        if cands:
            self.t = max(self.t, min(cands))

    def idle_wait(self):
        pass


def _requests(n, seed, rate, lo=20, hi=120):
    g = workloads.rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += float(g.exponential(1.0 / rate))
        w = int(g.choice([4, 8, 16]))
        m, n_ = int(g.integers(lo, hi)) + w, int(g.integers(lo, hi)) + w
        x, y = workloads.iid(g, m, workloads.DNA), workloads.iid(g, n_, workloads.DNA)
        out.append(serve.Request(k, x, y, w, workloads.DNA, threshold=(3 * w + 3) // 4, indel=True,
                                 arrival=t))
    return out


def test_budget_fifo_and_overlap(oracle_mod):
    reqs = _requests(60, 1, rate=400.0)
    budget = 6 * max(serve.footprint_bytes(r) for r in reqs)
    ex = FakeExecutor(oracle_mod, streams=2)
    srv = serve.Server(ex, budget_bytes=budget, max_jobs=10, max_batch=4)
    rep = srv.run(reqs)
    assert rep["rejected"] == 0 and rep["jobs"] == 60
    assert srv.peak_use <= budget
    # FIFO: admitted in arrival order
    order = [jid for _, jid in srv.admit_log]
    assert order == sorted(order)
    # continuous batching: some batch was launched while another was running
    assert any(running for _, _, running in ex.launch_log)
    assert srv.overlaps > 0
    # every job finished after it arrived, latencies are reported
    for js in srv.jobs.values():
        assert js.done >= js.launched >= js.admitted >= js.req.arrival
    assert rep["p99_s"] >= rep["p50_s"] > 0


def test_results_in_mix_equal_alone(oracle_mod):
    reqs = _requests(25, 2, rate=1000.0)
    srv = serve.Server(FakeExecutor(oracle_mod, streams=3), budget_bytes=1 << 40, max_batch=5)
    srv.run(reqs)
    for r in reqs:
        alone = oracle_mod.wlcs(r.x, r.y, r.w)
        res = srv.result(r.jid)
        np.testing.assert_array_equal(res["bitmap"], oracle_mod.dot_bitmap(alone, r.threshold))
        np.testing.assert_array_equal(res["indel"], oracle_mod.indel(alone, r.w))


def test_memory_pressure_holds_the_head(oracle_mod):
    # a budget that fits one job at a time: batches of one, strictly in order
    reqs = _requests(8, 3, rate=1e6)
    budget = max(serve.footprint_bytes(r) for r in reqs)
    ex = FakeExecutor(oracle_mod, streams=4)
    srv = serve.Server(ex, budget_bytes=budget)
    srv.run(reqs)
    assert srv.peak_use <= budget
    launches = sorted(srv.jobs.values(), key=lambda js: js.launched)
    assert [js.req.jid for js in launches] == list(range(8))
    # no two jobs were ever on the device together
    spans = sorted((js.launched, js.done) for js in srv.jobs.values())
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert b0 >= a1 - 1e-12


def test_oversized_job_is_rejected(oracle_mod):
    reqs = _requests(5, 4, rate=100.0)
    big = serve.Request(99, workloads.iid(workloads.rng(5), 5000, workloads.DNA),
                        workloads.iid(workloads.rng(6), 5000, workloads.DNA), 16, workloads.DNA,
                        threshold=12, arrival=0.001)
    budget = serve.footprint_bytes(big) - 1
    srv = serve.Server(FakeExecutor(oracle_mod), budget_bytes=budget)
    rep = srv.run(reqs + [big])
    assert rep["rejected"] == 1 and 99 in srv.rejected
    assert all(srv.poll(r.jid) for r in reqs)


def test_footprint_formula():
    r = serve.Request(0, np.zeros(1000, np.uint8), np.zeros(2000, np.uint8), 64, b"A", threshold=48,
                      indel=True, want_plot=True)
    rows, cols = 936, 1936
    want = 2 * 3000 + serve.PAIR_PAD_BYTES + rows * cols + rows * ((cols + 63) // 64) * 8 + rows * cols * 2
    assert serve.footprint_bytes(r) == want


def test_footprint_of_sparse_and_strided_jobs():
    x, y = np.zeros(1000, np.uint8), np.zeros(2000, np.uint8)
    r = serve.Request(0, x, y, 64, b"A", threshold=48, indel=False, hx=5, hy=2, dot_cap=5000)
    rows, cols = -(-936 // 5), -(-1936 // 2)
    assert serve.footprint_bytes(r) == 2 * 3000 + serve.PAIR_PAD_BYTES + 12 * 5000 + 8
    r = serve.Request(0, x, y, 64, b"A", threshold=48, indel=True, hx=5, hy=1)
    assert serve.footprint_bytes(r) == (2 * 3000 + serve.PAIR_PAD_BYTES + rows * ((1936 + 63) // 64) * 8
                                        + rows * 1936 * 2)
    assert serve.default_dot_cap(10, 10) == 4096 and serve.default_dot_cap(4096, 4096) == 262144


def test_sparse_jobs_results_equal_alone(oracle_mod):
    reqs = _requests(20, 6, rate=800.0)
    for k, r in enumerate(reqs):
        r.hx, r.hy = 1 + k % 3, 1 + (k // 3) % 2
        r.indel = False
        r.dot_cap = 10**6
    srv = serve.Server(FakeExecutor(oracle_mod, streams=2), budget_bytes=1 << 40, max_batch=4)
    rep = srv.run(reqs)
    assert rep["jobs"] == 20 and rep["rejected"] == 0
    for r in reqs:
        alone = oracle_mod.wlcs_strided(r.x, r.y, r.w, r.hx, r.hy)
        np.testing.assert_array_equal(srv.result(r.jid)["dots"],
                                      oracle_mod.dot_list(alone, r.w, r.threshold, r.hx, r.hy))


def test_short_dot_lists_are_rerun_complete(oracle_mod):
    """A job whose list overflows is rerun with room for every dot, ahead of
    later arrivals; its final list is complete."""
    reqs = _requests(12, 7, rate=500.0)
    for r in reqs:
        r.indel = False
        r.threshold = 0  # every window is a dot
        r.dot_cap = 5    # far too short
    srv = serve.Server(FakeExecutor(oracle_mod, streams=2), budget_bytes=1 << 40, max_batch=3)
    rep = srv.run(reqs)
    assert rep["rejected"] == 0 and rep["dot_list_reruns"] == 12
    for r in reqs:
        js = srv.jobs[r.jid]
        assert js.retries == 1 and js.done >= js.launched
        plot = oracle_mod.wlcs(r.x, r.y, r.w)
        assert srv.result(r.jid)["dot_count"] == plot.size
        np.testing.assert_array_equal(srv.result(r.jid)["dots"], oracle_mod.dot_list(plot, r.w, 0))


class SubBatchFakeExecutor(FakeExecutor):
    """Jobs of a batch finish one after another, cheapest first, each at its
    own time (as the GPU executor's sub-batches with their own events);
    poll_jobs reports them as they finish."""

    def launch(self, batch_id, jobs):
        super().launch(batch_id, jobs)  # results, and the stream taken
        k = next(i for i, b in enumerate(self.busy) if b is not None and b[1] == batch_id)
        t = self.t + self.overhead
        fins = []
        for j in sorted(jobs, key=serve.job_cost):
            t += float(j.req.x.size) * j.req.y.size * j.req.w / self.rate
            fins.append((t, j))
            j.fake_done = t
        self.busy[k] = (fins[-1][0], batch_id, fins)

    def poll_jobs(self):
        out = []
        for k, b in enumerate(self.busy):
            if b is None:
                continue
            fin = [j for t, j in b[2] if t <= self.t + 1e-12]
            rest = [(t, j) for t, j in b[2] if t > self.t + 1e-12]
            if fin or not rest:
                out.append((b[1], fin, not rest))
            self.busy[k] = (b[0], b[1], rest) if rest else None
        return out

    def advance(self, next_arrival):
        fins = [b[2][0][0] for b in self.busy if b is not None and b[2]]
        cands = fins + ([next_arrival] if next_arrival is not None else [])
        if cands:
            self.t = max(self.t, min(cands))


def test_jobs_complete_with_their_sub_batch(oracle_mod):
    """With per-job completion (poll_jobs) every job is done at its own finish
    time, its footprint is released then, results are unchanged, and the
    median latency is below that of whole-batch completion on the same
    stream of jobs."""
    reqs = _requests(60, 8, rate=400.0)
    budget = 6 * max(serve.footprint_bytes(r) for r in reqs)
    ex = SubBatchFakeExecutor(oracle_mod, streams=2)
    srv = serve.Server(ex, budget_bytes=budget, max_jobs=10, max_batch=4)
    rep = srv.run(reqs)
    assert rep["rejected"] == 0 and rep["jobs"] == 60
    assert srv.peak_use <= budget and srv.in_use == 0 and srv.active == 0 and not srv.running
    order = [jid for _, jid in srv.admit_log]
    assert order == sorted(order)
    for js in srv.jobs.values():
        assert js.done >= js.launched >= js.admitted >= js.req.arrival
        assert abs(js.done - js.fake_done) < 1e-9  # observed when it finished, not with its batch
        alone = oracle_mod.wlcs(js.req.x, js.req.y, js.req.w)
        np.testing.assert_array_equal(js.results["bitmap"], oracle_mod.dot_bitmap(alone, js.req.threshold))
    whole = serve.Server(FakeExecutor(oracle_mod, streams=2), budget_bytes=budget, max_jobs=10, max_batch=4)
    rep_whole = whole.run(_requests(60, 8, rate=400.0))
    assert rep["p50_s"] < rep_whole["p50_s"]


def test_sub_batch_reruns_of_short_dot_lists(oracle_mod):
    reqs = _requests(10, 9, rate=500.0)
    for r in reqs:
        r.indel = False
        r.threshold = 0
        r.dot_cap = 5
    srv = serve.Server(SubBatchFakeExecutor(oracle_mod, streams=2), budget_bytes=1 << 40, max_batch=3)
    rep = srv.run(reqs)
    assert rep["rejected"] == 0 and rep["dot_list_reruns"] == 10
    for r in reqs:
        plot = oracle_mod.wlcs(r.x, r.y, r.w)
        assert srv.result(r.jid)["dot_count"] == plot.size


# ---- failures forced from the host -------------------------------------

class OutOfMemoryError(RuntimeError):
    """What the device allocator raises when it has no memory left."""


class OomExecutor(FakeExecutor):
    """Fails a launch for lack of memory while `busy_limit` batches already
    run (an allocator that cannot hold more), or always when the batch holds
    one of the listed jobs."""

    def __init__(self, oracle, busy_limit=None, bad_jobs=(), **kw):
        super().__init__(oracle, **kw)
        self.busy_limit, self.bad_jobs = busy_limit, set(bad_jobs)
        self.failures = 0

    def launch(self, batch_id, jobs):
        running = sum(b is not None for b in self.busy)
        if any(j.req.jid in self.bad_jobs for j in jobs) or \
                (self.busy_limit is not None and running >= self.busy_limit):
            self.failures += 1
            raise OutOfMemoryError("out of memory (injected)")
        super().launch(batch_id, jobs)


def _check_results(srv, reqs, oracle_mod, statuses=("done",)):
    for r in reqs:
        js = srv.jobs[r.jid]
        if js.status != "done":
            continue
        plot = oracle_mod.wlcs(r.x, r.y, r.w)
        np.testing.assert_array_equal(srv.result(r.jid)["indel"], oracle_mod.indel(plot, r.w))


def test_out_of_memory_launch_waits_for_running_batches(oracle_mod):
    """A launch that finds no memory while other batches run puts its jobs
    back at the head of the queue; they run once memory is released, and
    every result equals the oracle's."""
    reqs = _requests(30, 91, rate=4000.0)
    ex = OomExecutor(oracle_mod, busy_limit=1, streams=3)
    srv = serve.Server(ex, budget_bytes=1 << 30, max_jobs=64, max_batch=4)
    rep = srv.run(reqs)
    assert ex.failures > 0 and rep["launch_retries"] > 0
    assert rep["failed"] == 0 and all(srv.status(r.jid) == "done" for r in reqs)
    assert srv.in_use == 0 and srv.active == 0
    _check_results(srv, reqs, oracle_mod)


def test_out_of_memory_with_nothing_running_fails_the_jobs(oracle_mod):
    """With no other batch to wait for, the jobs of a launch that finds no
    memory fail with the error recorded; the others are not affected and the
    budget is given back."""
    reqs = _requests(12, 92, rate=5.0)  # sparse arrivals: one batch at a time
    ex = OomExecutor(oracle_mod, bad_jobs={3})
    srv = serve.Server(ex, budget_bytes=1 << 30, max_jobs=64, max_batch=4)
    rep = srv.run(reqs)
    failed = [r.jid for r in reqs if srv.status(r.jid) == "failed"]
    assert failed and rep["failed"] == len(failed)
    assert all("out of memory" in srv.jobs[j].error for j in failed)
    assert all(srv.status(r.jid) in ("done", "failed") for r in reqs)
    assert srv.in_use == 0 and srv.active == 0
    _check_results(srv, reqs, oracle_mod)


class PartialExecutor(FakeExecutor):
    """Launches the first job of batch 1 and then runs out of memory."""

    def launch(self, batch_id, jobs):
        if batch_id == 1 and len(jobs) > 1:
            super().launch(batch_id, jobs[:1])
            raise serve.LaunchError(list(jobs[1:]), OutOfMemoryError("out of memory (injected)"))
        super().launch(batch_id, jobs)


def test_partly_launched_batch(oracle_mod):
    """A batch launched in part: the launched job completes with it, the rest
    return to the queue (another batch holds memory) and complete later."""
    reqs = _requests(24, 93, rate=1e9)
    for r in reqs:
        r.arrival = 0.0  # all at once: full batches of 4
    ex = PartialExecutor(oracle_mod, streams=3)
    srv = serve.Server(ex, budget_bytes=1 << 30, max_jobs=64, max_batch=4)
    rep = srv.run(reqs)
    assert rep["launch_retries"] == 3 and rep["failed"] == 0
    assert all(srv.status(r.jid) == "done" for r in reqs)
    assert srv.in_use == 0 and srv.active == 0
    _check_results(srv, reqs, oracle_mod)


def test_cancel_waiting_admitted_and_running_jobs(oracle_mod):
    reqs = _requests(10, 94, rate=1e9)  # all arrive at once
    ex = FakeExecutor(oracle_mod, streams=1)
    srv = serve.Server(ex, budget_bytes=1 << 30, max_jobs=64, max_batch=3)
    for r in reqs:
        srv.submit(r)
    srv.step()  # admits everything, launches the first batch of 3
    running = [js.req.jid for js in srv.running[0]]
    admitted = [js.req.jid for js in srv.admitted]
    assert len(running) == 3 and admitted
    assert srv.cancel(running[0]) and srv.cancel(admitted[0])
    assert not srv.cancel(running[0])  # already asked
    use_before = srv.in_use
    assert srv.status(admitted[0]) == "cancelled" and srv.in_use < use_before + 1
    while srv.busy():
        srv.step()
        ex.advance(None)
    assert srv.status(running[0]) == "cancelled" and srv.result(running[0]) is None
    assert srv.status(admitted[0]) == "cancelled"
    rep = srv.report()
    assert rep["cancelled"] == 2
    others = [r for r in reqs if r.jid not in (running[0], admitted[0])]
    assert all(srv.status(r.jid) == "done" for r in others)
    assert not srv.cancel(others[0].jid)  # already done
    assert srv.in_use == 0 and srv.active == 0
    _check_results(srv, others, oracle_mod)


def test_batch_timeout_on_the_virtual_clock(oracle_mod):
    """A batch that outruns the timeout has its jobs marked timed out (their
    results dropped, their memory released when the work ends); batches that
    finish in time are not affected."""
    reqs = _requests(16, 95, rate=20.0, lo=20, hi=60)
    big = reqs[5]
    big.x = np.concatenate([big.x] * 40)  # about 40x the work of the others
    ex = FakeExecutor(oracle_mod, streams=2, rate=2e6)
    srv = serve.Server(ex, budget_bytes=1 << 30, max_jobs=64, max_batch=1, batch_timeout_s=0.05)
    rep = srv.run(reqs)
    assert srv.status(big.jid) == "timed_out" and srv.result(big.jid) is None
    assert rep["timed_out"] >= 1
    assert all(srv.status(r.jid) in ("done", "timed_out") for r in reqs)
    assert sum(srv.status(r.jid) == "done" for r in reqs) >= 14
    assert srv.in_use == 0 and srv.active == 0
    _check_results(srv, reqs, oracle_mod)
