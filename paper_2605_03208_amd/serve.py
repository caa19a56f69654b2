"""Continuous-batching validation server.

A tuning agent submits validation requests: "compare these candidate outputs
of my reproducer against the captured goldens, with this ULP tolerance"
(the validation step of Sec. 4.5.2, and reproducers as a substrate for
tuning agents, Sec. 1 and Sec. 6).  Goldens stay resident on the device.

The loop:
  * requests arrive (Poisson schedule in the benchmark) into a FIFO queue;
  * the head of the queue is admitted when its candidate buffers fit in the
    HBM budget (head-of-line: a large request is never overtaken, so it
    cannot starve);
  * admitted requests are gathered into a batch as soon as a stream is free;
    the batch's candidates are materialised on that stream and all its pairs
    go to one persistent kc_compare launch, so requests that arrive while
    other batches are on the GPU overlap with them on the device;
  * completion is found by polling events; results are decoded, budget is
    returned, latency = result on host - scheduled arrival.

The executor is pluggable: ``DeviceExecutor`` runs on the GPU, ``MockExecutor``
runs the same admission / batching logic on the CPU for tests.
"""
from __future__ import annotations

import collections
import gc
import time
from dataclasses import dataclass, field

import numpy as np

DEFAULT_CLOSE = (1e-8, 1e-5)   # (atol, rtol) of the tolerance comparison, numpy.allclose's defaults


@dataclass
class Request:
    rid: int
    arrival_s: float
    golden_ids: np.ndarray
    ulp_tol: int
    seed: int


@dataclass
class Completed:
    rid: int
    arrival_s: float
    admit_s: float
    launch_s: float
    done_s: float
    nbytes: int
    results: list = field(default_factory=list)
    materialize_s: float = 0.0   # device time of the batch's candidate materialisation
    compare_s: float = 0.0       # device time of the batch's compare
    host_launch_s: float = 0.0   # host time spent issuing the batch (materialisation and compare calls)
    dev_start_s: float = 0.0     # device clock, from the start of the run: the batch's first and last event
    dev_end_s: float = 0.0

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class Budget:
    """Byte accounting of candidate buffers against the HBM budget."""

    def __init__(self, limit: int):
        self.limit = int(limit)
        self.used = 0
        self.peak = 0

    def try_take(self, n: int) -> bool:
        if self.used + n > self.limit:
            return False
        self.used += n
        self.peak = max(self.peak, self.used)
        return True

    def give(self, n: int) -> None:
        self.used -= n
        assert self.used >= 0


class MockExecutor:
    """CPU stand-in: a batch takes ``bytes / rate`` seconds of simulated time
    per stream; results are the request ids."""

    def __init__(self, sizes, n_streams: int = 2, rate_Bps: float = 1e12):
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.n_streams = n_streams
        self.rate = rate_Bps
        self.busy_until = [0.0] * n_streams
        self.batches = []

    def request_bytes(self, req: Request) -> int:
        return int(self.sizes[req.golden_ids].sum())

    def free_stream(self, now: float):
        for i, t in enumerate(self.busy_until):
            if t <= now and not any(b[0] == i for b in self.batches):
                return i
        return None

    def launch(self, stream: int, reqs, now: float):
        nbytes = sum(self.request_bytes(r) for r in reqs)
        self.busy_until[stream] = now + 2 * nbytes / self.rate
        h = (stream, reqs, self.busy_until[stream])
        self.batches.append(h)
        return h

    def done(self, h, now: float) -> bool:
        return now >= h[2]

    def finish(self, h):
        self.batches.remove(h)
        return [[dict(rid=r.rid)] for r in h[1]]


class DeviceExecutor:
    """Runs batches on ``n_streams`` HIP streams (one kc context each).  The
    goldens must be written by work already enqueued on the current stream
    when the executor is made (or finished): its streams wait for that work,
    since they do not order themselves after the current stream otherwise."""

    def __init__(self, goldens, dtypes, n_streams: int = 4, device=0, p_pert: float = 1e-4, kmax: int = 16,
                 arena_bytes: int | None = None):
        import torch

        from . import kc
        from . import workloads as W
        self.torch, self.kc, self.W = torch, kc, W
        self.goldens = goldens
        self.dtypes = [int(d) for d in dtypes]
        self.sizes = np.array([g.numel() * g.element_size() for g in goldens], dtype=np.int64)
        for g in goldens:
            assert g.is_cuda and g.is_contiguous(), "goldens must be contiguous device tensors"
        self.dtype_arr = np.array(self.dtypes, dtype=np.int64)
        self.numel_arr = np.array([g.numel() for g in goldens], dtype=np.int64)
        self.gold_ptr = np.array([g.data_ptr() for g in goldens], dtype=np.uint64)
        self.flat = [g.reshape(-1) for g in goldens]
        self.one_pass = bool(np.all(self.gold_ptr % np.uint64(16) == 0))  # kc_materialize needs 16-byte goldens
        self.n_elems_arr = self.sizes // np.array([kc.ELEM_SIZE[d] for d in self.dtypes], dtype=np.int64)
        self.n_streams = n_streams
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        # the goldens may still be being written on the current stream: a batch read them too early otherwise
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream(device))
        for st in self.streams:
            st.wait_event(ready)
        self.ctxs = [kc.Context(device) for _ in range(n_streams)]
        self.busy = [None] * n_streams
        self.arena_cache = {}  # stream -> byte buffer reused by that stream's batches
        self.arena_bytes = arena_bytes  # size of each stream's buffer when given (e.g. the server's budget)
        self.p_pert, self.kmax = p_pert, kmax
        self.block = max(1, int(round(1.0 / p_pert)))  # one moved element per block, as in W.perturb_many

    def request_bytes(self, req: Request) -> int:
        return int(self.sizes[req.golden_ids].sum())

    def free_stream(self, now: float):
        for i, b in enumerate(self.busy):
            if b is None:
                return i
        return None

    def candidate_seed(self, req: Request, gid: int) -> int:
        return (int(req.seed) * 1000003 + int(gid)) & 0x7FFFFFFF

    def launch(self, stream: int, reqs, now: float):
        """Materialise the batch's candidates (per element type: one
        kc_materialize launch that copies and moves the goldens into a fresh
        arena, or a copy and a kc_perturb launch where a golden is not 16-byte
        aligned) and run all its pairs in one kc_compare launch.  The pair
        list is built from arrays of addresses (no tensor per pair), in
        request order."""
        torch, kc = self.torch, self.kc
        s = self.streams[stream]
        counts = np.array([len(r.golden_ids) for r in reqs], dtype=np.int64)
        gids = np.concatenate([np.asarray(r.golden_ids, dtype=np.int64) for r in reqs])
        # candidate_seed, vectorised: (seed * 1000003 + gid) mod 2^31 with the product reduced first
        base = np.array([(int(r.seed) * 1000003) & 0x7FFFFFFF for r in reqs], dtype=np.int64)
        seeds = (np.repeat(base, counts) + gids) & 0x7FFFFFFF
        dts = self.dtype_arr[gids]
        cand_ptr = np.zeros(len(gids), dtype=np.uint64)
        ev0, ev_mat, ev = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        arenas = []
        # one arena per element type, carved from the stream's buffer at 256-byte aligned byte offsets
        plan, total = [], 0
        for dt in np.unique(dts):
            sel = np.nonzero(dts == dt)[0]
            lens = self.numel_arr[gids[sel]]
            esz = self.flat[int(gids[sel[0]])].element_size()
            align = max(1, 16 // esz)   # keep every candidate 16-byte aligned
            padded = -(-lens // align) * align
            plan.append((sel, lens, esz, padded, total))
            total += -(-int(padded.sum()) * esz // 256) * 256
        with torch.cuda.stream(s):
            ev0.record(s)
            buf = self.arena(stream, total)
            for sel, lens, esz, padded, at in plan:
                golds = [self.flat[g] for g in gids[sel].tolist()]
                offs = np.concatenate([[0], np.cumsum(padded)[:-1]]).astype(np.int64)
                arena = buf[at: at + int(padded.sum()) * esz].view(golds[0].dtype)
                if self.one_pass:
                    kc.materialize(self.ctxs[stream], arena, self.gold_ptr[gids[sel]], offs, lens, seeds[sel],
                                   self.block, self.kmax, stream=s)
                else:
                    if np.array_equal(padded, lens):
                        torch.cat(golds, out=arena)
                    else:
                        for g, o, n in zip(golds, offs.tolist(), lens.tolist()):
                            arena[o: o + n].copy_(g)
                    kc.perturb(self.ctxs[stream], arena, offs, lens, seeds[sel], self.block, self.kmax, stream=s)
                arenas.append(arena)
                cand_ptr[sel] = np.uint64(arena.data_ptr()) + offs.astype(np.uint64) * np.uint64(esz)
            pairs = kc.pairs_from_arrays(cand_ptr, self.gold_ptr[gids], self.n_elems_arr[gids], dts,
                                         np.repeat([int(r.ulp_tol) for r in reqs], counts), *DEFAULT_CLOSE)
            ev_mat.record(s)
            res = kc.compare(self.ctxs[stream], pairs)
            ev.record(s)
        h = dict(stream=stream, reqs=reqs, res=res, ev=ev, ev0=ev0, ev_mat=ev_mat, arenas=arenas, n=len(gids),
                 owners=np.repeat([r.rid for r in reqs], counts).tolist())
        self.busy[stream] = h
        return h

    def arena(self, stream: int, nbytes: int):
        """The candidate bytes of a batch on ``stream``: a view of one buffer
        per stream, reused since a stream runs one batch at a time.  With
        ``arena_bytes`` each buffer is made that size on first use (a server
        passes its budget, which bounds any batch); otherwise it grows in whole
        GiB to the largest batch seen, an outgrown buffer going back to the
        device (a synchronising free).  Fresh device allocations of budget-sized
        arenas in every batch stalled the loop for up to a second now and then
        (the allocator's retry path)."""
        buf = self.arena_cache.get(stream)
        need = max(256, nbytes)
        if buf is None or buf.numel() < need:
            self.arena_cache[stream] = None
            if buf is not None:  # hand the outgrown buffer back to the device rather than to torch's cache
                del buf
                self.torch.cuda.empty_cache()
            grain = 1 << 30
            size = max(-(-need // grain) * grain, self.arena_bytes or 0)
            buf = self.torch.empty(size, dtype=self.torch.uint8, device=self.streams[stream].device)
            self.arena_cache[stream] = buf
        return buf[:need]

    def done(self, h, now: float) -> bool:
        return h["ev"].query()

    def begin(self) -> None:
        """Marks the start of a run on the device clock (a reference event that
        every batch's events are timed against)."""
        self.ref = self.torch.cuda.Event(enable_timing=True)
        self.ref.record(self.streams[0])

    def split(self, h) -> tuple:
        """(materialise, compare) device seconds of a finished batch."""
        return h["ev0"].elapsed_time(h["ev_mat"]) / 1e3, h["ev_mat"].elapsed_time(h["ev"]) / 1e3

    def interval(self, h) -> tuple:
        """(start, end) of a finished batch on the device, in seconds from begin()."""
        return self.ref.elapsed_time(h["ev0"]) / 1e3, self.ref.elapsed_time(h["ev"]) / 1e3

    def finish(self, h):
        out = self.kc.decode_cmp(h["res"], h["n"])
        self.busy[h["stream"]] = None
        per = collections.defaultdict(list)
        for rid, r in zip(h["owners"], out):
            per[rid].append(r)
        return [per[r.rid] for r in h["reqs"]]


class Server:
    def __init__(self, executor, budget_bytes: int, max_batch: int = 64, clock=None, sleep=None):
        self.ex = executor
        self.budget = Budget(budget_bytes)
        self.max_batch = max_batch
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.admit_order = []

    def run(self, requests, real_time: bool = True, poll_s: float = 50e-6):
        """Serve ``requests`` (sorted by arrival).  Returns Completed records
        in completion order.  Python's cyclic garbage collector is paused
        while the loop runs (a full collection over the results of earlier
        runs stalls the loop for tens of milliseconds); reference counting
        still frees every batch's buffers as it completes."""
        was_enabled = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, real_time, poll_s)
        finally:
            if was_enabled:
                gc.enable()

    def _run(self, requests, real_time: bool, poll_s: float):
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        for r in reqs:
            if self.ex.request_bytes(r) > self.budget.limit:
                raise ValueError(f"request {r.rid} needs more than the whole budget")
        pending = collections.deque(reqs)
        queue = collections.deque()
        admitted = []          # (req, admit_s)
        running = []           # (handle, [(req, admit_s)], launch_s, host_launch_s)
        done = []
        if hasattr(self.ex, "begin"):
            self.ex.begin()
        t0 = self.clock()
        now = 0.0
        while pending or queue or admitted or running:
            now = self.clock() - t0 if real_time else now
            while pending and pending[0].arrival_s <= now:
                queue.append(pending.popleft())
            while queue and self.budget.try_take(self.ex.request_bytes(queue[0])):
                r = queue.popleft()
                admitted.append((r, now))
                self.admit_order.append(r.rid)
            progressed = False
            while admitted:
                st = self.ex.free_stream(now)
                if st is None:
                    break
                batch, admitted = admitted[: self.max_batch], admitted[self.max_batch:]
                t_issue = self.clock()
                h = self.ex.launch(st, [r for r, _ in batch], now)
                running.append((h, batch, now, self.clock() - t_issue if real_time else 0.0))
                progressed = True
            still = []
            for h, batch, t_launch, host_s in running:
                if self.ex.done(h, now):
                    results = self.ex.finish(h)
                    t_done = self.clock() - t0 if real_time else now
                    mat_s, cmp_s = self.ex.split(h) if hasattr(self.ex, "split") else (0.0, 0.0)
                    d0, d1 = self.ex.interval(h) if hasattr(self.ex, "interval") else (0.0, 0.0)
                    for (r, t_adm), res in zip(batch, results):
                        self.budget.give(self.ex.request_bytes(r))
                        done.append(Completed(r.rid, r.arrival_s, t_adm, t_launch, t_done,
                                              self.ex.request_bytes(r), res, mat_s, cmp_s, host_s, d0, d1))
                    progressed = True
                else:
                    still.append((h, batch, t_launch, host_s))
            running = still
            if not progressed:
                if real_time:
                    nxt = pending[0].arrival_s - now if pending and not (queue or admitted or running) else poll_s
                    self.sleep(max(0.0, min(nxt, 1e-3)))
                else:
                    # simulated time: jump to the next event
                    cands = [pending[0].arrival_s] if pending else []
                    cands += [h[2] for h, _, _, _ in running if isinstance(h, tuple)]
                    nxt = min([c for c in cands if c > now], default=now + poll_s)
                    now = nxt
        return done


def summarize(done, wall_s: float) -> dict:
    """Latency percentiles, split into queue (arrival to admission), wait
    (arrival to the start of its batch's launch), the host time of issuing
    the batch, and the device time of the materialisation and the compare of
    each request's batch; aggregate compared bytes (both sides) per second;
    the device-busy fraction: the union of the batches' device intervals
    (first event to last, over all streams) divided by the wall time."""
    def pct(values, p):
        return round(float(np.percentile(np.array(values) if values else np.zeros(1), p)) * 1e3, 3)

    lat = [d.latency_s for d in done]
    q = [d.admit_s - d.arrival_s for d in done]
    wait = [d.launch_s - d.arrival_s for d in done]
    host = [d.host_launch_s for d in done]
    mat = [d.materialize_s for d in done]
    cmp_ = [d.compare_s for d in done]
    nbytes = sum(2 * d.nbytes for d in done)
    busy, end = 0.0, float("-inf")
    for a, b in sorted({(d.dev_start_s, d.dev_end_s) for d in done}):
        if b > end:
            busy += b - max(a, end)
            end = b
    return dict(requests=len(done), p50_ms=pct(lat, 50), p99_ms=pct(lat, 99),
                queue_p50_ms=pct(q, 50), queue_p99_ms=pct(q, 99),
                wait_p50_ms=pct(wait, 50), wait_p99_ms=pct(wait, 99),
                host_launch_p50_ms=pct(host, 50), host_launch_p99_ms=pct(host, 99),
                materialize_p50_ms=pct(mat, 50), materialize_p99_ms=pct(mat, 99),
                compare_p50_ms=pct(cmp_, 50), compare_p99_ms=pct(cmp_, 99),
                aggregate_GBps=round(nbytes / max(wall_s, 1e-9) / 1e9, 1), compared_bytes=nbytes,
                busy_frac=round(busy / max(wall_s, 1e-9), 4), wall_s=round(wall_s, 3))
