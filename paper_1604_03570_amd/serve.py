"""Continuous-batching server of independent periodic heat problems.

Requests (domain edge n, box edge, step count, FP32 or FP64) arrive over time.
The loop:

* admits them while slots and the HBM budget allow, strictly first come first
  served: a request that does not fit holds back those behind it, so large ones
  cannot starve;
* allocates their MultiFab pair in HBM and loads the initial field;
* lets every admitted request join the next tick of one shared Batch;
* advances every member by one step per tick: one fused FillBoundary+stencil
  launch per dtype over all members' tiles, the paper's collapsed (grid, tile)
  loop of Sec. 3.3 spanning every problem;
* issues several ticks per pass of the loop (Batch.steps), as many as no member
  finishes before the last of them and at most max_steps, so the loop's host
  work is paid once per pass, not once per step; the host runs at most
  max_ahead_steps steps ahead of the GPU, which bounds how long a request that
  arrives meanwhile waits to join;
* retires a request, freeing its memory, when its step count is reached.

Latency is completion minus arrival. Completion is the GPU time of the event
recorded after the request's last step, mapped to the host clock.

All numerical work runs in libboxtile's kernels. torch provides only device
memory, the stream and the events, plus the elementwise product that
expands a separable initial field (input synthesis, not the method).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import boxtile as bt
from . import inputs as I


# ----------------------------------------------------------------------------- admission
@dataclass
class Admission:
    """First-come-first-served admission under a slot limit and an HBM byte budget."""
    budget: int
    max_slots: int
    used: int = 0
    active: int = 0

    def admit(self, queue: deque, footprint) -> list:
        """Pop and return the requests at the head of `queue` that fit now, in order;
        stop at the first that does not.  A request larger than the whole budget can
        never fit and is rejected (returned with footprint None) so the queue moves."""
        out = []
        while queue and self.active < self.max_slots:
            r = queue[0]
            need = footprint(r)
            if need > self.budget:
                queue.popleft()
                out.append((r, None))
                continue
            if self.used + need > self.budget:
                break
            queue.popleft()
            self.used += need
            self.active += 1
            out.append((r, need))
        return out

    def release(self, nbytes: int) -> None:
        self.used -= nbytes
        self.active -= 1
        assert self.used >= 0 and self.active >= 0


# ----------------------------------------------------------------------------- problems
_DT = {"f64": bt.F64, "f32": bt.F32}


class _Shapes:
    """BoxArrays per (domain edge, box edge), so MultiFabs of one shape share a plan."""

    def __init__(self):
        self._ba = {}

    def boxarray(self, n: int, box_edge: int) -> bt.BoxArray:
        key = (n, box_edge)
        if key not in self._ba:
            self._ba[key] = bt.BoxArray.chop(I.domain_box(n), min(box_edge, n))
        return self._ba[key]

    def footprint(self, r: I.Request) -> int:
        """HBM bytes of a request's two MultiFabs (1 component, 1 ghost)."""
        return 2 * self.boxarray(r.n, r.box_edge).multifab_bytes(1, 1, _DT[r.dtype])


def initial_field(r: I.Request, device=None) -> torch.Tensor:
    """The request's Gaussian bump u0 = 1 + (gz (x) gy) (x) gx, expanded from its three
    1-D factors (inputs.gaussian_factors) on `device`, FP64, shape (1, n, n, n)."""
    gx, gy, gz = (torch.as_tensor(v, device=device) for v in I.gaussian_factors(r.n, r.center))
    return (1.0 + (gz[:, None, None] * gy[None, :, None]) * gx[None, None, :])[None]


@dataclass
class _Live:
    req: I.Request
    mid: int
    a: bt.MultiFab
    b: bt.MultiFab
    nbytes: int
    joined_tick: int
    admit_host: float


@dataclass
class ServeStats:
    completed: int = 0
    rejected: int = 0
    ticks: int = 0
    launches: int = 0      # passes of the loop that issued steps (Batch.steps calls)
    host_us: list = field(default_factory=list)    # host time of each such pass, admission to bookkeeping,
                                                   # without the time spent waiting for the GPU
    launch_us: list = field(default_factory=list)  # of which in Batch.steps (the launches themselves)
    latencies_ms: list = field(default_factory=list)
    queue_ms: list = field(default_factory=list)
    cell_updates: int = 0
    makespan_s: float = 0.0
    peak_bytes: int = 0
    peak_active: int = 0
    mean_active: float = 0.0

    def summary(self) -> dict:
        lat = np.asarray(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        q = np.asarray(self.queue_ms) if self.queue_ms else np.zeros(1)
        return {
            "completed": self.completed, "rejected": self.rejected, "ticks": self.ticks,
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "max_ms": round(float(lat.max()), 3),
            "queue_p50_ms": round(float(np.percentile(q, 50)), 3), "queue_p99_ms": round(float(np.percentile(q, 99)), 3),
            "throughput_gcell_s": round(self.cell_updates / max(self.makespan_s, 1e-9) / 1e9, 3),
            "makespan_s": round(self.makespan_s, 3), "peak_hbm_bytes": self.peak_bytes,
            "peak_active": self.peak_active, "mean_active": round(self.mean_active, 2),
            "launches": self.launches, "steps_per_launch": round(self.ticks / max(self.launches, 1), 2),
            "host_us_per_launch_p50": round(float(np.percentile(self.host_us, 50)), 1) if self.host_us else 0.0,
            "launch_us_per_launch_p50": round(float(np.percentile(self.launch_us, 50)), 1) if self.launch_us else 0.0,
        }


class Server:
    """Runs a request stream against one GPU in real time (arrival times are honoured
    on the host clock).  `on_complete(req, result_tensor)` receives each finished
    request's final field (dense (1, n, n, n) device tensor) when given."""

    def __init__(self, hbm_budget: int, max_slots: int = 64, max_steps: int = 16, max_ahead_steps: int = 16,
                 on_complete=None):
        self.adm = Admission(int(hbm_budget), int(max_slots))
        self.max_steps = max(1, int(max_steps))
        self.max_ahead_steps = max(1, int(max_ahead_steps))
        self.on_complete = on_complete
        self.shapes = _Shapes()

    def prepare(self, requests) -> None:
        """Make every problem shape of the stream resident ahead of time, as in a
        long-running server: its device tables, its kernels loaded (those that build an
        initial field too) and the allocator holding blocks of its size, by admitting one
        problem per shape as a request would be and one batched step."""
        seen = set()
        batch = bt.Batch()
        keep = []
        for r in requests:
            key = (r.n, r.box_edge, r.dtype)
            if key in seen:
                continue
            seen.add(key)
            ba = self.shapes.boxarray(r.n, r.box_edge)
            a, b = bt.MultiFab(ba, 1, 1, _DT[r.dtype]), bt.MultiFab(ba, 1, 1, _DT[r.dtype])
            a.from_global(initial_field(r, device=a.buffer.device))
            keep.append((a, b, batch.add(a, b, I.heat_c(r.n))))
        if keep:
            batch.step()
            torch.cuda.synchronize()
            for _, _, mid in keep:
                batch.remove(mid)
        del keep, batch
        torch.cuda.synchronize()

    def run(self, requests, stream=None, prepare: bool = True) -> ServeStats:
        assert torch.cuda.is_available(), "the server needs a GPU"
        stream = stream or torch.cuda.current_stream()
        if prepare:
            self.prepare(requests)
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue = deque()
        live = {}
        batch = bt.Batch()
        st = ServeStats()
        done_events = []       # (event, request)
        ahead = deque()        # (event, steps) of recent launches, to bound host run-ahead
        ahead_steps = 0
        active_sum = 0
        tick = 0
        with torch.cuda.stream(stream):
            torch.cuda.synchronize()
            t0_ev = torch.cuda.Event(enable_timing=True)
            t0_ev.record(stream)
            t0 = time.perf_counter()
            while pending or queue or live:
                h0 = time.perf_counter()
                now = h0 - t0
                while pending and pending[0].arrival <= now:
                    queue.append(pending.popleft())
                for r, need in self.adm.admit(queue, self.shapes.footprint):
                    if need is None:
                        st.rejected += 1
                        continue
                    ba = self.shapes.boxarray(r.n, r.box_edge)
                    a = bt.MultiFab(ba, 1, 1, _DT[r.dtype])
                    b = bt.MultiFab(ba, 1, 1, _DT[r.dtype])
                    a.from_global(initial_field(r, device=a.buffer.device), stream=stream)
                    mid = batch.add(a, b, I.heat_c(r.n))
                    live[mid] = _Live(r, mid, a, b, need, tick, now)
                    st.queue_ms.append((now - r.arrival) * 1e3)
                st.peak_bytes = max(st.peak_bytes, self.adm.used)
                st.peak_active = max(st.peak_active, len(live))
                if not live:
                    if pending:
                        time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.002)))
                    continue
                k = min(self.max_steps, min(L.req.steps - (tick - L.joined_tick) for L in live.values()))
                l0 = time.perf_counter()
                batch.steps(k, stream)
                l1 = time.perf_counter()
                tick += k
                st.launches += 1
                active_sum += len(live) * k
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(stream)
                ahead.append((ev, k))
                ahead_steps += k
                w0 = time.perf_counter()
                while ahead_steps - ahead[-1][1] >= self.max_ahead_steps:  # keep the newest launch in flight
                    e_old, k_old = ahead.popleft()
                    e_old.synchronize()
                    ahead_steps -= k_old
                waited = time.perf_counter() - w0
                finished = [m for m, L in live.items() if tick - L.joined_tick == L.req.steps]
                for m in finished:
                    L = live.pop(m)
                    cur = L.a if L.req.steps % 2 == 0 else L.b
                    if self.on_complete is not None:
                        self.on_complete(L.req, cur.to_global(stream=stream))
                    batch.remove(m)
                    self.adm.release(L.nbytes)
                    done_events.append((ev, L.req))
                    st.cell_updates += L.req.n ** 3 * L.req.steps
                st.launch_us.append((l1 - l0) * 1e6)
                st.host_us.append((time.perf_counter() - h0 - waited) * 1e6)  # without waiting on the GPU
            torch.cuda.synchronize()
            last = 0.0
            for ev, r in done_events:
                t_done = t0_ev.elapsed_time(ev) / 1e3
                st.latencies_ms.append((t_done - r.arrival) * 1e3)
                last = max(last, t_done)
            st.completed = len(done_events)
            st.ticks = tick
            first = min((r.arrival for r in requests), default=0.0)
            st.makespan_s = last - first
            st.mean_active = active_sum / max(tick, 1)
        return st


def serve_stream(requests, hbm_budget: int, max_slots: int = 64, on_complete=None, **kw) -> dict:
    return Server(hbm_budget, max_slots, on_complete=on_complete, **kw).run(requests).summary()


def offered_load(requests) -> float:
    """Cell updates per second the stream asks for (sum of n^3 * steps over its span)."""
    if not requests:
        return 0.0
    span = max(r.arrival for r in requests) - min(r.arrival for r in requests)
    return sum(r.n ** 3 * r.steps for r in requests) / max(span, 1e-9)


__all__ = ["Admission", "Server", "ServeStats", "initial_field", "serve_stream", "offered_load"]
