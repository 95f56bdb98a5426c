"""Streaming service: continuous batching of filterbank chunks from many streams.

Requests (one chunk of packed time-major rows of one stream) arrive at any
time.  A scheduler thread admits them under a device-memory budget, groups
the admitted head-of-line chunks of distinct streams into a *tick*, copies
them to the device on a copy stream, and enqueues the tick as one batched
launch (``dedisp_stream_push_many``: one corner-turn launch for all chunks, then a single
multi-beam kernel over every chunk's tiles) on the compute stream, without
waiting for earlier ticks: new requests are admitted while others are on the
GPU and their work overlaps there.  A completion thread waits for each tick's
event, stamps every request's completion time and releases its memory, which
lets waiting requests in.

Each stream keeps its last max_delay rows on the device (its history), so the
outputs of a stream's requests, concatenated, are the one-shot transform of
its concatenated input; a request's output does not depend on which other
requests share its tick.

Latency = completion of the request's outputs on the device minus its
arrival time (host clock).  Output tensors stay on the device; the caller
receives them in the finished Request, or in an ``on_done`` callback run by
the completion thread as each request finishes (a consumer that drops the
output there lets the device allocator reuse its memory for later ticks).
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

QUEUED, RUNNING, DONE, REJECTED, FAILED, CANCELLED = (
    "queued", "running", "done", "rejected", "failed", "cancelled")


@dataclass
class Request:
    stream_id: int
    seq: int
    data: np.ndarray              # packed rows, uint8 [nsamps][row_bytes]
    t_arrival: float
    status: str = QUEUED
    reason: str = ""
    t_admit: float = 0.0
    t_launch: float = 0.0
    t_done: float = 0.0
    n_out: int = 0
    out: object = None            # device tensor [ndm][>= n_out] (int32 holding uint32 sums)
    nbytes: int = 0
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def nsamps(self) -> int:
        return int(self.data.shape[0])

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class GpuExecutor:
    """Runs ticks on the GPU through the library's streams (one per service stream)."""

    def __init__(self, plans, device="cuda:0", max_chunk: int | None = None):
        """max_chunk: longest chunk any request will carry; when given, every
        stream's scratch is sized for it up front (and again after tune()), so
        no push has to grow it -- growing frees the old scratch, which waits
        for the whole device and drains the ticks queued behind it."""
        import torch
        from .api import Stream
        self.torch = torch
        self.device = torch.device(device)
        self.plans = list(plans)
        self.streams = [Stream(p) for p in self.plans]
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.compute_stream = torch.cuda.Stream(device=self.device)
        self.max_chunk = max_chunk
        self._reserve()

    def _reserve(self):
        if self.max_chunk:
            for s in self.streams:
                s.reserve(self.max_chunk)

    def tune(self, nsamps: int, cache_path: str | None = None):
        """Pick each distinct plan's tile shape by timing the candidates on a
        zero chunk of `nsamps` rows (the integer sums take the same time
        whatever the data).  Streams read their plan's shape at every push, so
        later ticks use the tuned shapes."""
        torch = self.torch
        seen = set()
        for p in self.plans:
            if id(p) in seen:
                continue
            seen.add(id(p))
            n = max(int(nsamps), p.max_delay + 1)
            inp = torch.zeros(n * p.row_bytes, dtype=torch.uint8, device=self.device)
            out = torch.empty((p.ndm, n - p.max_delay), dtype=torch.int32, device=self.device)
            p.tune(inp, out, n, cache_path=cache_path)
            del inp, out
        torch.cuda.synchronize(self.device)
        self._reserve()

    def request_bytes(self, stream_id: int, nsamps: int) -> int:
        """Device bytes a request holds while admitted: its chunk and its outputs."""
        p = self.plans[stream_id]
        return nsamps * p.row_bytes + p.ndm * nsamps * 4

    def resident_bytes(self) -> int:
        """Device bytes held whatever is admitted: every stream's history and
        channel-major scratch (as reserved for max_chunk)."""
        return sum(s.device_bytes() for s in self.streams)

    def launch(self, reqs):
        """Enqueue one tick; returns an object whose wait() blocks until it is done."""
        torch = self.torch
        from .api import push_many
        chunks, outs = [], []
        with torch.cuda.stream(self.copy_stream):
            for r in reqs:
                host = torch.from_numpy(np.ascontiguousarray(r.data).reshape(-1))
                if not host.is_pinned():
                    host = host.pin_memory()
                dev = torch.empty(host.numel(), dtype=torch.uint8, device=self.device)
                dev.copy_(host, non_blocking=True)
                chunks.append(dev)
                p = self.plans[r.stream_id]
                outs.append(torch.empty((p.ndm, r.nsamps), dtype=torch.int32, device=self.device))
        copied = torch.cuda.Event()
        copied.record(self.copy_stream)
        self.compute_stream.wait_event(copied)
        with torch.cuda.stream(self.compute_stream):
            n_outs = push_many([self.streams[r.stream_id] for r in reqs], chunks, outs,
                               out_row_strides=[r.nsamps for r in reqs],
                               stream=self.compute_stream)
            for t in chunks + outs:
                t.record_stream(self.compute_stream)
        done = torch.cuda.Event()
        done.record(self.compute_stream)
        for r, o, n in zip(reqs, outs, n_outs):
            r.out, r.n_out = o, n
        return done

    @staticmethod
    def wait(handle):
        handle.synchronize()


class Server:
    """Admission, per-stream ordering and continuous batching (see module docstring)."""

    def __init__(self, executor, nstreams: int, budget_bytes: int, max_tick: int = 16,
                 max_inflight_ticks: int = 4, admit_timeout_s: float | None = None,
                 on_done=None):
        self.ex = executor
        self.on_done = on_done
        self._in_callbacks = 0                    # finished ticks whose callbacks still run
        self._launching = 0                       # ticks taken from the queues, not yet in flight
        self.callback_errors = []                 # (request, repr of what on_done raised)
        self.nstreams = int(nstreams)
        # The budget bounds all device memory of the service: what the streams
        # hold between requests (history and scratch) is charged up front, the
        # rest is shared by the admitted requests.
        self.total_budget = int(budget_bytes)
        self.resident = 0
        self.budget = 0
        self._charge_resident()
        self.max_tick = int(max_tick)
        self.max_inflight = int(max_inflight_ticks)
        self.admit_timeout = admit_timeout_s
        self.used = 0
        self.peak_used = 0
        self.fifo = [collections.deque() for _ in range(self.nstreams)]
        self.next_seq = [0] * self.nstreams
        self.inflight = collections.deque()       # (handle, [requests])
        self.finished = []
        self.ticks = 0
        self.tick_sizes = []
        self._lock = threading.Condition()
        self._stop = False
        self._threads = []

    def _charge_resident(self):
        res = getattr(self.ex, "resident_bytes", None)
        self.resident = int(res()) if res is not None else 0
        self.budget = self.total_budget - self.resident
        if self.budget <= 0:
            raise ValueError(f"the streams' resident device memory ({self.resident} bytes) "
                             f"leaves nothing of the {self.total_budget}-byte budget")

    # -------------------------------------------------------------- client
    def submit(self, stream_id: int, data: np.ndarray, seq: int | None = None,
               t_arrival: float | None = None) -> Request:
        """Queue one chunk of stream `stream_id`; chunks of a stream must come in order."""
        now = time.perf_counter() if t_arrival is None else t_arrival
        with self._lock:
            want = self.next_seq[stream_id]
            req = Request(stream_id, want if seq is None else int(seq), data, now)
            if not (0 <= stream_id < self.nstreams):
                return self._reject(req, "unknown stream")
            if req.seq != want:
                return self._reject(req, f"out-of-order chunk: expected {want}, got {req.seq}")
            if data.ndim != 2 or data.dtype != np.uint8 or data.shape[0] == 0:
                return self._reject(req, "malformed chunk")
            req.nbytes = self.ex.request_bytes(stream_id, data.shape[0])
            if req.nbytes > self.budget:
                return self._reject(req, "chunk larger than the memory budget")
            self.next_seq[stream_id] += 1
            self.fifo[stream_id].append(req)
            self._lock.notify_all()
            return req

    def cancel(self, req: Request) -> bool:
        """Cancel a request that has not been admitted yet."""
        with self._lock:
            q = self.fifo[req.stream_id]
            if req.status == QUEUED and req in q:
                q.remove(req)
                req.status = CANCELLED
                req.done.set()
                self.finished.append(req)
                self._lock.notify_all()
                return True
            return False

    def start(self):
        # the executor may have re-reserved its streams' scratch (tuning)
        with self._lock:
            self._charge_resident()
        self._threads = [threading.Thread(target=self._schedule, daemon=True),
                         threading.Thread(target=self._complete, daemon=True)]
        for t in self._threads:
            t.start()
        return self

    def drain(self, timeout: float | None = None):
        """Wait until every submitted request has finished."""
        t_end = None if timeout is None else time.perf_counter() + timeout
        with self._lock:
            while any(self.fifo) or self.inflight or self._launching or self._in_callbacks:
                left = None if t_end is None else t_end - time.perf_counter()
                if left is not None and left <= 0:
                    raise TimeoutError("drain timed out")
                self._lock.wait(0.05 if left is None else min(0.05, left))

    def stop(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        for t in self._threads:
            t.join()

    # ------------------------------------------------------------- threads
    def _reject(self, req, why):
        req.status, req.reason = REJECTED, why
        req.done.set()
        self.finished.append(req)
        return req

    def _pick_tick(self):
        """Head-of-line chunks of distinct streams, oldest first, within the budget."""
        heads = [q[0] for q in self.fifo if q]
        heads.sort(key=lambda r: r.t_arrival)
        tick = []
        now = time.perf_counter()
        for r in heads:
            if len(tick) >= self.max_tick:
                break
            if self.used + r.nbytes > self.budget:
                if self.admit_timeout is not None and now - r.t_arrival > self.admit_timeout:
                    self.fifo[r.stream_id].popleft()
                    self._reject(r, "memory budget: admission timed out")
                continue
            self.fifo[r.stream_id].popleft()
            self.used += r.nbytes
            self.peak_used = max(self.peak_used, self.used)
            r.status, r.t_admit = RUNNING, now
            tick.append(r)
        return tick

    def _schedule(self):
        while True:
            with self._lock:
                while not self._stop and (not any(self.fifo)
                                          or len(self.inflight) >= self.max_inflight):
                    self._lock.wait(0.01)
                if self._stop:
                    return
                tick = self._pick_tick()
                if not tick:
                    self._lock.wait(0.001)
                    continue
                self._launching += 1
            t_launch = time.perf_counter()
            try:
                handle = self.ex.launch(tick)
                err = None
            except Exception as e:                  # the tick fails, its memory is released
                handle, err = None, e
            with self._lock:
                self._launching -= 1
                for r in tick:
                    r.t_launch = t_launch
                if err is not None:
                    for r in tick:
                        r.status, r.reason = FAILED, repr(err)
                        self.used -= r.nbytes
                        r.out = None
                        r.done.set()
                        self.finished.append(r)
                else:
                    self.inflight.append((handle, tick))
                    self.ticks += 1
                    self.tick_sizes.append(len(tick))
                self._lock.notify_all()

    def _complete(self):
        while True:
            with self._lock:
                while not self._stop and not self.inflight:
                    self._lock.wait(0.01)
                if self._stop and not self.inflight:
                    return
                handle, tick = self.inflight[0]
            self.ex.wait(handle)
            t_done = time.perf_counter()
            with self._lock:
                self.inflight.popleft()
                for r in tick:
                    r.t_done = t_done
                    r.status = DONE
                    self.used -= r.nbytes
                    self.finished.append(r)
                self._in_callbacks += 1
                self._lock.notify_all()
            # outside the lock: the callback may take its time
            try:
                for r in tick:
                    if self.on_done is not None:
                        try:
                            self.on_done(r)
                        except Exception as e:      # a failing consumer must not stop the server
                            with self._lock:
                                self.callback_errors.append((r, repr(e)))
                    r.done.set()
            finally:
                with self._lock:
                    self._in_callbacks -= 1
                    self._lock.notify_all()

    # ------------------------------------------------------------- metrics
    def stats(self):
        done = [r for r in self.finished if r.status == DONE]
        lat = np.array([r.latency for r in done]) if done else np.zeros(1)
        return {
            "requests_done": len(done),
            "rejected": sum(r.status == REJECTED for r in self.finished),
            "failed": sum(r.status == FAILED for r in self.finished),
            "cancelled": sum(r.status == CANCELLED for r in self.finished),
            "ticks": self.ticks,
            "mean_tick_size": float(np.mean(self.tick_sizes)) if self.tick_sizes else 0.0,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_max_s": float(lat.max()),
            "peak_budget_bytes": self.peak_used,
            "resident_bytes": self.resident,
            "peak_device_bytes": self.resident + self.peak_used,
            "budget_bytes": self.total_budget,
        }
