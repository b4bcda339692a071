"""Continuous-batching request loop over resident imaging jobs.

Requests (PSF-convolution applies, degrid, grid, FAST likelihood gradients and
20-iteration CG solves) arrive on a recorded Poisson trace.  The loop

  * keeps every job's plan, PSF kernels and data resident on the device;
  * coalesces pending requests of the same job and operation into one batched
    launch (up to `max_batch`, batchable operations only);
  * admits a launch only while the sum of the per-call scratch footprints in
    flight (fr_query_footprint) stays within the HBM budget and a stream is free;
  * runs launches of different jobs concurrently on a pool of streams (default
    priority) and detects completion with events, so new arrivals are admitted as
    soon as slots and memory free up;
  * records arrival -> completion latency per request;
  * drops cancelled requests: one cancelled while pending (its t_cancel has
    passed, or Server.cancel was called from another thread) is never launched;
    one cancelled while on the device keeps its slot and memory until the launch
    finishes (device work is not preempted), then frees both and its result is
    discarded.

The scheduling logic is independent of the GPU: an executor object launches a
batch and reports whether it has finished.  `GpuExecutor` drives libfrmi through
`api`; tests use a simulated executor on the CPU.
"""

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

OPS = ("psf_apply", "degrid", "grid", "lik_fast", "cg20")
BATCHABLE = {"psf_apply", "lik_fast"}
DEFAULT_MIX = {"psf_apply": 0.35, "degrid": 0.15, "grid": 0.15, "lik_fast": 0.20, "cg20": 0.15}


@dataclass
class Request:
    rid: int
    t_arrival: float
    job: int
    op: str
    size: int = 1          # images in the request (PSF apply, likelihood samples)
    t_release: float = None  # when the loop saw it (= arrival in real time)
    t_start: float = None
    t_done: float = None
    batch: int = 0         # number of requests it was launched with
    t_cancel: float = None  # the client gives up at this trace time (None: never)
    cancelled: bool = False


@dataclass
class Launch:
    job: int
    op: str
    reqs: list
    bytes: int
    handle: object = None
    slot: int = -1


def make_trace(n_jobs, rate_hz, duration_s, seed=240609148, mix=None, max_size=8):
    """Poisson arrivals (exponential gaps) with the operation mix; returns Requests."""
    mix = mix or DEFAULT_MIX
    rng = np.random.default_rng(seed)
    ops = list(mix)
    p = np.array([mix[o] for o in ops], dtype=float)
    p /= p.sum()
    t, reqs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        op = ops[rng.choice(len(ops), p=p)]
        size = int(rng.integers(1, max_size + 1)) if op == "lik_fast" else 1
        reqs.append(Request(len(reqs), t, int(rng.integers(0, n_jobs)), op, size))
    return reqs


class Server:
    """Continuous batching with footprint admission over an executor."""

    def __init__(self, executor, n_slots=4, hbm_budget=64 << 30, max_batch=8, clock=time.perf_counter):
        self.ex = executor
        self.n_slots = n_slots
        self.budget = hbm_budget
        self.max_batch = max_batch
        self.clock = clock
        self.peak_bytes = 0
        self.launches = []
        self.free_slots = list(range(n_slots))
        self.bytes_in_flight = 0
        self._cancel_lock = threading.Lock()
        self._cancel_ids = set()

    def cancel(self, rid):
        """Cancel request `rid` (thread-safe; takes effect at the loop's next turn)."""
        with self._cancel_lock:
            self._cancel_ids.add(rid)

    def _is_cancelled(self, r, now):
        if r.t_cancel is not None and r.t_cancel <= now:
            return True
        with self._cancel_lock:
            return r.rid in self._cancel_ids

    def _form_batches(self, pending):
        """Group pending requests by (job, op), oldest group first."""
        groups = collections.OrderedDict()
        for r in pending:
            groups.setdefault((r.job, r.op), []).append(r)
        out = []
        for (job, op), rs in groups.items():
            if op in BATCHABLE:
                cur, n = [], 0
                for r in rs:
                    if cur and n + r.size > self.max_batch:
                        out.append((job, op, cur))
                        cur, n = [], 0
                    cur.append(r)
                    n += r.size
                if cur:
                    out.append((job, op, cur))
            else:
                out.extend((job, op, [r]) for r in rs)
        out.sort(key=lambda g: g[2][0].t_arrival)
        return out

    def run(self, trace, realtime=True):
        """Serve `trace` (sorted by arrival).  With realtime, arrivals are released at
        their trace times relative to the start; otherwise all at once."""
        trace = sorted(trace, key=lambda r: r.t_arrival)
        t0 = self.clock()
        nxt = 0
        pending = []
        inflight = []
        free_slots = self.free_slots = list(range(self.n_slots))
        used = 0
        done = 0
        while done < len(trace):
            now = self.clock() - t0
            while nxt < len(trace) and (not realtime or trace[nxt].t_arrival <= now):
                trace[nxt].t_release = now
                pending.append(trace[nxt])
                nxt += 1
            # cancelled while waiting: never launched
            keep = []
            for r in pending:
                if self._is_cancelled(r, now):
                    r.cancelled = True
                    r.t_done = now
                    done += 1
                else:
                    keep.append(r)
            pending = keep
            # completions free slots and memory
            still = []
            for L in inflight:
                if self.ex.done(L.handle):
                    tdone = self.clock() - t0
                    for r in L.reqs:
                        r.t_done = tdone
                        r.cancelled = self._is_cancelled(r, tdone)
                    used -= L.bytes
                    free_slots.append(L.slot)
                    done += len(L.reqs)
                else:
                    still.append(L)
            inflight = still
            self.bytes_in_flight = used
            # admission
            if pending and free_slots:
                launched = set()
                for job, op, rs in self._form_batches(pending):
                    if not free_slots:
                        break
                    B = sum(r.size for r in rs)
                    nbytes = self.ex.footprint(job, op, B)
                    if nbytes > self.budget:
                        raise RuntimeError(f"request ({job}, {op}, B={B}) exceeds the HBM budget on its own")
                    if used + nbytes > self.budget:
                        continue
                    slot = free_slots.pop(0)
                    L = Launch(job, op, rs, nbytes, slot=slot)
                    tstart = self.clock() - t0
                    for r in rs:
                        r.t_start = tstart
                        r.batch = len(rs)
                    L.handle = self.ex.launch(job, op, rs, slot)
                    used += nbytes
                    self.peak_bytes = max(self.peak_bytes, used)
                    inflight.append(L)
                    self.launches.append((job, op, len(rs), B, nbytes))
                    launched.update(id(r) for r in rs)
                pending = [r for r in pending if id(r) not in launched]
            elif not inflight and not pending and nxt < len(trace) and realtime:
                time.sleep(max(0.0, min(1e-3, trace[nxt].t_arrival - (self.clock() - t0))))
        return trace


def latency_stats(reqs, from_release=False):
    """Latency percentiles from arrival (or from release, for traces replayed
    without their arrival times) to completion, over the requests not cancelled."""
    reqs = [r for r in reqs if not r.cancelled]
    t0 = [r.t_release if from_release else r.t_arrival for r in reqs]
    lat = np.array([r.t_done - t for r, t in zip(reqs, t0)])
    span = max(r.t_done for r in reqs) - min(t0)
    return {"n": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "throughput_req_s": len(reqs) / span if span > 0 else float("nan")}


# ---------------------------------------------------------------------- GPU executor
@dataclass
class ServedJob:
    plan: object
    psf: object
    vis: object        # data visibilities [n_row, 1]
    weight: object     # [n_row, 1]
    dirty: object      # [1, n, n]
    inv_power: object  # [n, n/2 + 1]
    images: object     # pool of input images [P, 1, n, n]
    logsky: object     # pool of log-sky samples [P, 1, n, n]
    outputs: dict = field(default_factory=dict)


class GpuExecutor:
    """Launches batches through libfrmi on a pool of streams (default priority).
    With timeline=True every launch is bracketed by timing events on its stream,
    so that the device intervals of the launches (and their overlap across
    streams) can be read back after the run (`timeline_intervals`)."""

    def __init__(self, jobs, n_slots=4, keep_outputs=False, timeline=False):
        import torch
        from . import api
        self.api = api
        self.torch = torch
        self.jobs = jobs
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.keep = keep_outputs
        self.results = {}
        self.timeline = [] if timeline else None
        self._t_ref = None
        if timeline:
            torch.cuda.synchronize()
            self._t_ref = torch.cuda.Event(enable_timing=True)
            self._t_ref.record()
        from ._lib import FR_OP_CG, FR_OP_DEGRID, FR_OP_GRID, FR_OP_LIK_FAST, FR_OP_RNR_APPROX
        self.opcode = {"psf_apply": FR_OP_RNR_APPROX, "degrid": FR_OP_DEGRID, "grid": FR_OP_GRID,
                       "lik_fast": FR_OP_LIK_FAST, "cg20": FR_OP_CG}

    def footprint(self, job, op, B):
        J = self.jobs[job]
        s, _ = self.api.query_footprint(self.opcode[op], B, plan=J.plan if op in ("degrid", "grid") else None,
                                        psf=J.psf if op not in ("degrid", "grid") else None)
        n = J.plan.nx * J.plan.ny
        io = 4 * n * B * 2 + (8 * J.plan.n_row if op in ("degrid",) else 0)  # inputs gathered + outputs
        return s + io

    def _input(self, pool, r, k):
        return pool[(r.rid + k) % pool.shape[0]]

    def launch(self, job, op, reqs, slot):
        torch, api = self.torch, self.api
        from ._lib import FR_LIK_FAST
        J = self.jobs[job]
        st = self.streams[slot]
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            if self.timeline is not None:
                e_start = torch.cuda.Event(enable_timing=True)
                e_start.record(st)
            if op == "psf_apply":
                x = torch.stack([self._input(J.images, r, k) for r in reqs for k in range(r.size)])
                y = api.apply_RNR_approx(J.psf, x, stream=st)
                outs = self._split(y, reqs)
            elif op == "lik_fast":
                s = torch.stack([self._input(J.logsky, r, k) for r in reqs for k in range(r.size)])
                H, g = api.likelihood_grad(FR_LIK_FAST, s, J.dirty, psf=J.psf, inv_power=J.inv_power, stream=st)
                outs = self._split(g, reqs)
            elif op == "degrid":
                outs = [api.degrid(J.plan, self._input(J.images, reqs[0], 0), stream=st)]
            elif op == "grid":
                outs = [api.grid(J.plan, J.vis, J.weight, stream=st)]
            else:
                x, hist, it = api.cg_solve(self._input(J.images, reqs[0], 0), psf=J.psf, inv_power=J.inv_power,
                                           maxiter=20, stream=st)
                outs = [x]
            if self.timeline is not None:
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(st)
                self.timeline.append((slot, op, e_start, ev))
            else:
                ev = torch.cuda.Event()
                ev.record(st)
        if self.keep:
            for r, o in zip(reqs, outs):
                self.results[r.rid] = o
        return (ev, outs)

    @staticmethod
    def _split(t, reqs):
        outs, k = [], 0
        for r in reqs:
            outs.append(t[k:k + r.size])
            k += r.size
        return outs

    def done(self, handle):
        return handle[0].query()

    def timeline_intervals(self):
        """(slot, op, start_ms, end_ms) of every launch, device time from the
        executor's creation (call after the stream work has finished)."""
        self.torch.cuda.synchronize()
        return [(slot, op, self._t_ref.elapsed_time(a), self._t_ref.elapsed_time(b))
                for slot, op, a, b in self.timeline]


def overlap_stats(intervals):
    """Device-side concurrency of launch intervals (start, end) on several streams:
    the summed launch time, the time at least one launch was running, their ratio
    (> 1 when launches of different streams ran together) and the largest number
    running at once."""
    if not intervals:
        return {"launches": 0}
    ev = sorted([(a, 1) for a, b in intervals] + [(b, -1) for a, b in intervals])
    busy, cur, peak, last = 0.0, 0, 0, None
    for t, d in ev:
        if cur > 0 and last is not None:
            busy += t - last
        cur += d
        peak = max(peak, cur)
        last = t
    total = sum(b - a for a, b in intervals)
    return {"launches": len(intervals), "launch_ms_sum": total, "busy_ms": busy,
            "concurrency": total / busy if busy > 0 else float("nan"), "max_concurrent": peak}
