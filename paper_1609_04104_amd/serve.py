"""Continuous-batching server for many concurrent scans on one GPU.

Scans arrive over time; each streams k-space frames at a fixed rate.  A scan is
admitted when the device pool has room for its resident state
(``tsl_open_in_pool``); over budget it waits, first come first served.  Every
turn of the loop takes, from every admitted scan whose next frame has arrived,
that frame, and launches them together as one batched step (``tsl_step_many``,
which groups them by shape).  Frames that arrive while a step is on the GPU
join a later step, so the batch follows the load.  After its warm frames a scan
acquires the rows that its previous step drew on the device (Algorithm 4), so no
frame waits for the host to see the previous one's result.

The latency of a frame is the device completion time of its step minus the
frame's arrival time.  ``plain=True`` serves the same arrivals one frame at a
time (``tsl_push_frame`` in arrival order), the single-sequence baseline.

This module only schedules: every step of the method runs in libtsl.
"""

import time

import numpy as np
import torch

from . import tsl


class Scan:
    """One acquisition: shape, rank, initial factors, a bank of full k-space
    frames on the device (frame t acquires rows of bank[t % len(bank)]), the
    number of frames, arrival time (s) and frame rate (frames/s)."""

    def __init__(self, sid, n, r, lam, A0, B0, bank, T, arrival, fps, t_warm=5, K=None, seed=1609,
                 record=False):
        self.sid, self.n, self.r, self.lam = sid, n, r, lam
        self.A0, self.B0, self.bank = A0, B0, bank
        self.T, self.arrival, self.fps, self.t_warm = T, arrival, fps, t_warm
        self.K = K if K else max(1, n // 8)
        self.seed = seed
        # record=True keeps every frame's output and every drawn row set on the
        # device (X_hist [T][n][n], rows_hist [T+1][K], cnt_hist [T+1]) instead of
        # reusing one output and two row buffers
        self.record = record
        self.seq = None
        self.t = 0            # frames launched
        self.done = 0         # frames completed
        self.admitted_at = None
        self._frames = {}

    def frame_arrival(self, t):
        return self.arrival + t / self.fps

    def open(self, pool, stream):
        dev = self.bank.device
        self.seq = tsl.Sequence(self.n, self.n, self.r, self.lam, self.A0, self.B0, seed=self.seed,
                                stream_id=self.sid, pool=pool, stream=stream)
        self.rows = [torch.zeros(self.K, dtype=torch.int32, device=dev) for _ in range(2)]
        self.cnt = [torch.zeros(1, dtype=torch.int32, device=dev) for _ in range(2)]
        self.full = torch.arange(self.n, dtype=torch.int32, device=dev)
        self.X = torch.empty(self.n, self.n, dtype=torch.complex64, device=dev)
        if self.record:
            self.X_hist = torch.empty(self.T, self.n, self.n, dtype=torch.complex64, device=dev)
            self.rows_hist = torch.zeros(self.T + 1, self.K, dtype=torch.int32, device=dev)
            self.cnt_hist = torch.zeros(self.T + 1, 1, dtype=torch.int32, device=dev)

    def next_frame(self):
        t = self.t
        if self.record:
            y = self.bank[t % self.bank.shape[0]]
            nxt = dict(K_next=self.K, rows_next=self.rows_hist[t + 1], n_next=self.cnt_hist[t + 1])
            if t < self.t_warm:
                return self.seq.frame(rows=self.full, y=y, y_full=True, X_out=self.X_hist[t], **nxt)
            return self.seq.frame(rows=self.rows_hist[t], n_rows_dev=self.cnt_hist[t], y=y, y_full=True,
                                  X_out=self.X_hist[t], **nxt)
        key = (t % self.bank.shape[0], t % 2, t < self.t_warm)
        f = self._frames.get(key)
        if f is None:
            y = self.bank[key[0]]
            nxt = dict(K_next=self.K, rows_next=self.rows[(t + 1) % 2], n_next=self.cnt[(t + 1) % 2])
            if key[2]:
                f = self.seq.frame(rows=self.full, y=y, y_full=True, X_out=self.X, **nxt)
            else:
                f = self.seq.frame(rows=self.rows[t % 2], n_rows_dev=self.cnt[t % 2], y=y, y_full=True,
                                   X_out=self.X, **nxt)
            self._frames[key] = f
        return f

    def close(self):
        if self.seq is not None:
            self.seq.close()
            self.seq = None
        self._frames = {}


class _Events:
    """Recycled timing events."""

    def __init__(self):
        self.free = []

    def get(self):
        return self.free.pop() if self.free else torch.cuda.Event(enable_timing=True)

    def put(self, e):
        self.free.append(e)


def serve(scans, budget_bytes, stream=None, plain=False, max_inflight=4, max_batch=1024, time_limit=None,
          on_finish=None):
    """Runs every scan to completion (or until time_limit seconds of wall time)
    and returns frame counts, throughput and latency percentiles.  on_finish(scan)
    is called after a scan's last frame completed, before its state is freed."""
    stream = stream or torch.cuda.current_stream()
    pool = tsl.Pool(budget_bytes)
    pending = sorted(scans, key=lambda s: s.arrival)
    waiting, active = [], []
    inflight = []                     # (event, [(scan, t)])
    events = _Events()
    lat, batch_sizes, admit_wait = [], [], []
    n_frames = 0
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last_done = 0.0

    def retire(block):
        nonlocal n_frames, last_done
        while inflight:
            ev, items = inflight[0]
            if not block and not ev.query():
                return
            ev.synchronize()
            done = ev0.elapsed_time(ev) * 1e-3
            last_done = max(last_done, done)
            for sc, t in items:
                lat.append(done - sc.frame_arrival(t))
                sc.done += 1
                n_frames += 1
                if sc.done == sc.T:
                    if on_finish is not None:
                        on_finish(sc)
                    sc.close()
                    active.remove(sc)
            events.put(ev)
            inflight.pop(0)
            block = False

    try:
        while pending or waiting or active:
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                break
            while pending and pending[0].arrival <= now:
                waiting.append(pending.pop(0))
            while waiting:
                sc = waiting[0]
                try:
                    sc.open(pool, stream)
                except tsl.TslError as e:
                    if e.code != tsl.EBUSY:
                        raise
                    break
                sc.admitted_at = now
                admit_wait.append(now - sc.arrival)
                active.append(sc)
                waiting.pop(0)
            ready = [sc for sc in active if sc.t < sc.T and sc.frame_arrival(sc.t) <= now]
            if plain:
                ready.sort(key=lambda sc: sc.frame_arrival(sc.t))
                ready = ready[:1]
            else:
                ready = ready[:max_batch]
            if ready:
                while len(inflight) >= max_inflight:
                    retire(True)
                items = []
                if plain:
                    sc = ready[0]
                    sc.seq.push(sc.next_frame(), stream)
                    items.append((sc, sc.t))
                    sc.t += 1
                else:
                    frames = [sc.next_frame() for sc in ready]
                    tsl.step_many([sc.seq for sc in ready], frames, stream)
                    for sc in ready:
                        items.append((sc, sc.t))
                        sc.t += 1
                ev = events.get()
                ev.record(stream)
                inflight.append((ev, items))
                batch_sizes.append(len(items))
            else:
                retire(False)
                if not inflight:
                    # nothing on the device: sleep until the next arrival
                    nxt = [sc.frame_arrival(sc.t) for sc in active if sc.t < sc.T]
                    if pending:
                        nxt.append(pending[0].arrival)
                    if nxt:
                        dt = min(nxt) - (time.perf_counter() - t0)
                        if dt > 0:
                            time.sleep(min(dt, 0.002))
        retire(True)
    finally:
        for sc in scans:
            sc.close()
        pool.destroy()
    lat = np.asarray(lat)
    first = min(sc.arrival for sc in scans) if scans else 0.0
    span = max(last_done - first, 1e-9)
    return {
        "frames": int(n_frames),
        "frames_per_s": n_frames / span,
        "span_s": span,
        "latency_p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
        "latency_p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
        "latency_max_ms": float(lat.max() * 1e3) if lat.size else None,
        "mean_batch": float(np.mean(batch_sizes)) if batch_sizes else 0.0,
        "steps": len(batch_sizes),
        "admit_wait_p99_ms": float(np.percentile(admit_wait, 99) * 1e3) if admit_wait else None,
    }
