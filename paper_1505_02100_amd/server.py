"""Continuous-batching bandwidth-selection server (Python front end).

The scheduling engine is native (kde_server_* in libkdeplugin): admission into
slots against a device-memory budget, resident samples, and steps that each
launch the persistent kernel over the next work items of every active request.
This module keeps the Python-side bookkeeping: the arrival queue of a trace,
the lifetime of device sample tensors, and latency statistics.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import kdeplugin as kp
from . import synth


@dataclass
class Completion:
    id: int
    n: int
    h: float
    status: int
    psi6: float
    psi4: float
    t_submit_ms: float
    t_admit_ms: float
    t_done_ms: float
    arrival_s: Optional[float] = None
    dist: Optional[str] = None
    seed: Optional[int] = None

    @property
    def latency_ms(self) -> float:
        return self.t_done_ms - self.t_submit_ms


class Server:
    """Owns a kde_server on a context; keeps submitted device tensors alive
    until their request completes."""

    def __init__(self, ctx: "kp.Context", mem_budget: int = 8 << 30, max_active: int = 64,
                 step_pairs: int = 1 << 34, policy: str = "fcfs", aging_ms: int = 0, fill: str = "share"):
        o = kp.kde_server_options_init()
        o.mem_budget = int(mem_budget)
        o.max_active = int(max_active)
        o.step_pairs = int(step_pairs)
        o.policy = {"fcfs": kp.KDE_SERVE_FCFS, "sjf": kp.KDE_SERVE_SJF}[policy]
        o.aging_ms = int(aging_ms)
        o.fill = {"share": kp.KDE_FILL_SHARE, "priority": kp.KDE_FILL_PRIORITY}[fill]
        self.ctx = ctx
        self.options = o
        self.handle = kp.kde_server_create(ctx.handle, o)
        self._keep: Dict[int, object] = {}

    def close(self):
        if self.handle:
            kp.kde_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, x) -> int:
        s = kp._Samples(x)
        if s.dtype != kp.KDE_F64:
            raise TypeError("server samples must be float64")
        # a device tensor's producer is torch's current stream on its device
        rid = kp.kde_server_submit(self.handle, s.ptr, s.n, s.mem, s.stream)
        self._keep[rid] = s.keep
        return rid

    def cancel(self, rid: int) -> None:
        kp.kde_server_cancel(self.handle, rid)
        self._keep.pop(rid, None)

    def step(self, block: bool = False) -> kp.kde_server_stats:
        return kp.kde_server_step(self.handle, block)

    def poll(self) -> List[Completion]:
        out = []
        for c in kp.kde_server_poll(self.handle):
            self._keep.pop(c.id, None)
            r = c.result
            out.append(Completion(c.id, c.n, r.h, r.status, r.psi6, r.psi4, c.t_submit_ms, c.t_admit_ms,
                                  c.t_done_ms))
        return out

    def drain(self) -> List[Completion]:
        kp.kde_server_drain(self.handle)
        return self.poll()

    def fail_next_step(self, code: int = kp.KDE_EDEVICE) -> None:
        kp.kde_server_fail_next_step(self.handle, code)


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else math.nan


def sjf_key(n: int, waited_s: float, aging_s: float) -> float:
    """Smallest-first key with aging, as the native admission uses it: log2 of
    the pair count minus one per aging_s of waiting (aging_s = 0: none)."""
    k = math.log2(max(1.0, float(n) * (n - 1)))
    return k - waited_s / aging_s if aging_s > 0 else k


def serve_trace(ctx: "kp.Context", trace, duration_s: float, mem_budget: int = 8 << 30,
                max_active: int = 64, step_pairs: int = 1 << 34, policy: str = "fcfs",
                aging_ms: int = 0, fill: str = "share", lookahead: int = 8, drain: bool = False,
                device: str = "cuda",
                keep_samples: bool = False, log=None) -> dict:
    """Replay `trace` (list of (arrival_s, n, dist, seed), sorted by arrival) in
    wall-clock time for `duration_s` seconds.  A request is drawn on the
    device (synth.draw_torch) and submitted when it has arrived and the
    server has room for it (at most `lookahead` submitted but not yet
    admitted); later arrivals wait in a host queue, as they would at a front
    end, in arrival order (FCFS) or by the aged smallest-first key (SJF).
    Latency is measured from the arrival time (the server's timestamps and
    time.monotonic() share the host's monotonic clock).  With drain, the loop
    goes on after the window until every arrived request has finished.

    The backlog at the end gives the pair evaluations still owed to
    unfinished requests and the time the device would take to drain them at
    the rate it ran during the loop (a full drain at a heavy overload runs for
    many minutes).

    Reported over ALL arrivals, not only the completed ones: a request still
    unfinished when the loop stops counts at its elapsed time (a lower bound
    on its latency), so the percentiles are lower bounds whenever that many
    requests are unfinished ("censored").  The served rate counts the pair
    evaluations of completed requests; the pair evaluations the device
    issued (including partial work on unfinished requests) are reported
    beside it.  With keep_samples the device samples of completed requests
    are returned too."""
    import torch
    srv = Server(ctx, mem_budget=mem_budget, max_active=max_active, step_pairs=step_pairs, policy=policy,
                 aging_ms=aging_ms, fill=fill)
    aging_s = aging_ms / 1e3
    pending = list(trace)
    pending.reverse()                    # pop() from the end = earliest arrival
    waiting: List = []                   # arrived, not yet submitted
    meta: Dict[int, tuple] = {}          # submitted, not yet completed
    samples: Dict[int, object] = {}
    done: List[Completion] = []
    t0 = time.monotonic()
    offered_pairs = 0.0
    arrived = 0
    last_log = 0.0
    while True:
        now = time.monotonic() - t0
        while pending and pending[-1][0] <= min(now, duration_s):
            a = pending.pop()
            waiting.append(a)
            offered_pairs += a[1] * (a[1] - 1)
            arrived += 1
        stats = srv.step(block=False)
        # submit arrived requests while the server has room for them
        if policy == "sjf":
            waiting.sort(key=lambda a: sjf_key(a[1], now - a[0], aging_s))
        while waiting and stats.queued < lookahead and stats.active + stats.queued < max_active:
            a = waiting.pop(0)
            x = synth.draw_torch(a[2], a[1], a[3], device=device)
            rid = srv.submit(x)
            meta[rid] = a
            if keep_samples:
                samples[rid] = x
            stats = srv.step(block=False)
        for c in srv.poll():
            c.arrival_s, _, c.dist, c.seed = meta.pop(c.id)
            done.append(c)
        if log is not None and now - last_log > 5.0:
            last_log = now
            log(f"t={now:6.1f}s arrived={arrived} done={len(done)} active={stats.active} "
                f"waiting={len(waiting)} steps={stats.steps}")
        if now >= duration_s and not drain:
            break
        if now >= duration_s and drain and not waiting and stats.active == 0 and stats.queued == 0:
            break
        if not waiting and stats.active == 0 and stats.queued == 0 and not pending:
            break
        if stats.inflight_steps >= 1 and not waiting:
            srv.step(block=True)
    window = time.monotonic() - t0
    end_ms = (t0 + window) * 1e3
    stats = srv.step(block=False)
    for c in srv.poll():
        c.arrival_s, _, c.dist, c.seed = meta.pop(c.id)
        done.append(c)
    issued = stats.pairs_issued
    failed_steps = stats.failed_steps
    srv.close()
    lat_done = [c.t_done_ms - (t0 + c.arrival_s) * 1e3 for c in done]
    unfinished = list(waiting) + list(meta.values())
    lat_open = [end_ms - (t0 + a[0]) * 1e3 for a in unfinished]
    lat_all = lat_done + lat_open
    served = sum(c.n * (c.n - 1) for c in done if c.status == 0)
    # pair evaluations still owed at the end: the unfinished requests' totals
    # less the partial work the device already issued for them
    owed = sum(a[1] * (a[1] - 1) for a in unfinished)
    partial = max(0.0, issued - sum(c.n * (c.n - 1) for c in done))
    remaining = max(0.0, owed - partial)
    issued_rate = issued / window if window > 0 else 0.0

    def pct(v):
        return {"p50": percentile(v, 50), "p99": percentile(v, 99), "max": max(v) if v else math.nan}

    def censored(q):
        # an unfinished request's latency is at least its elapsed time, so the
        # q-th percentile over all arrivals is exact when every unfinished
        # request already lies at or above it, and a lower bound otherwise
        if not lat_all or not lat_open:
            return False
        return min(lat_open) < percentile(lat_all, q)

    # per size decade: arrivals, completions and the all-arrivals median
    by_size = []
    for lo, hi in ((1e3, 1e4), (1e4, 1e5), (1e5, 1e6), (1e6, 1e7)):
        ld = [l for c, l in zip(done, lat_done) if lo <= c.n < hi]
        lo_ = [l for a, l in zip(unfinished, lat_open) if lo <= a[1] < hi]
        by_size.append({"n_from": int(lo), "n_to": int(hi), "arrived": len(ld) + len(lo_), "completed": len(ld),
                        "p50_ms_all": percentile(ld + lo_, 50),
                        "p50_is_lower_bound": bool(lo_) and min(lo_) < percentile(ld + lo_, 50)})

    return {"completions": done, "window_s": window, "arrived": arrived,
            "offered_pair_evals_per_s": offered_pairs / max(duration_s, 1e-9),
            "completed_pair_evals_per_s": served / window,
            "device_pair_evals_per_s": issued / window,
            "selections_per_s": len(done) / window,
            "latency_ms": pct(lat_done),
            "latency_ms_all_arrivals": dict(pct(lat_all), p50_is_lower_bound=censored(50),
                                            p99_is_lower_bound=censored(99)),
            "unfinished": len(unfinished),
            "by_size": by_size,
            "failed": sum(1 for c in done if c.status != 0),
            "failed_steps": failed_steps,
            "backlog": {"waiting": len(waiting), "active": len(meta) - stats.queued, "queued": stats.queued,
                        "not_arrived": len(pending), "remaining_pair_evals": remaining,
                        "drain_s_at_device_rate": remaining / issued_rate if issued_rate > 0 else math.nan},
            "samples": samples}
