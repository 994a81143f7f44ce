#!/usr/bin/env python3
"""Throughput and latency of the online PARAFAC tracking step on one MI355X.

Workload (synthetic cardiac-like cine; the paper's in-vivo scans are not
available): S sequences of N x N frames (default 64 x 256^2), rank R = 32,
lambda = 0.05, MM step size.  Every sequence starts with 5 fully sampled frames
(warm start) and then acquires the rows that the previous step drew on the
device (Algorithm 4, row score of Sec. VI-C, K = N/8 draws with replacement).
One step = one frame of every sequence through the whole hot path: partial
Grams, ridge solve and step size, synthesis + row transform, column transform +
residual + column inverse, row inverse + gradients, factor updates with their
k-space transforms, the output frame X_t, and the next rows -- all inputs
resident in HBM before the timed region.

Prints one JSON line: batched frames/s (value), the plain single-sequence path
on the same GPU, p50/p99 per-frame latency of both, the per-phase split, the
roofline of the dominant kernel and the FP64 CPU oracle's frames/s.
"""

import argparse
import gc
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--seqs", type=int, default=64)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--r", type=int, default=32)
    ap.add_argument("--lam", type=float, default=0.05)
    ap.add_argument("--frames", type=int, default=25, help="distinct k-space frames per sequence (cycled)")
    ap.add_argument("--plain-frames", type=int, default=200)
    ap.add_argument("--phase-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--procs", type=int, default=16, help="host processes generating the inputs (1: in-process)")
    ap.add_argument("--bank-frames", type=int, default=16, help="distinct frames per shape, mixed and served legs")
    ap.add_argument("--mixed-steps", type=int, default=50)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--serve-scans", type=int, default=128)
    ap.add_argument("--serve-rate", type=float, default=16.0, help="scan arrivals per second at load 1")
    ap.add_argument("--serve-T", type=int, default=150, help="frames per scan")
    ap.add_argument("--serve-loads", type=str, default="1,8,32",
                    help="offered-load factors: arrival rate and frame rate (30/s) both times the factor")
    ap.add_argument("--serve-limit", type=float, default=20.0, help="wall-time cap per served run (s)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--mall-seqs", type=int, default=1024,
                    help="sequences of the leg whose frame arrays overflow the 256 MB Infinity Cache (0: skip)")
    ap.add_argument("--mall-steps", type=int, default=10)
    ap.add_argument("--route", choices=["kspace", "frame"], default="kspace",
                    help="line-mask route of the headline measurement")
    ap.add_argument("--frame-route-steps", type=int, default=20,
                    help="steps of the same batch on the frame route (0: skip that leg)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a known-size "
                         "reference for hardware byte counters)")
    return ap.parse_args()


# ----------------------------------------------------------------------------- inputs
def _gen(args):
    n, r, frames, seq = args
    from paper_1609_04104_amd import inputs as I
    c = I.config3_kspace(T=frames, n1=n, n2=n, r=r, seq=seq)
    return c["kspace"], c["A0"], c["B0"]


def make_inputs(seqs, n, r, frames, procs=16):
    procs = max(1, min(procs, os.cpu_count() or 1, seqs))
    jobs = [(n, r, frames, s) for s in range(seqs)]
    if procs == 1:
        return [_gen(j) for j in jobs]
    with mp.get_context("spawn").Pool(procs) as pool:
        return pool.map(_gen, jobs)


# ----------------------------------------------------------------------------- work model
def phase_work(n1, n2, r, rows, K, kspace=True):
    """Algorithmic bytes, flops and arithmetic kind per frame of each phase
    (complex64 = 8 B, complex128 = 16 B, complex MAC = 8 flop, length-N complex
    FFT = 5 N log2 N flop).  Bytes are the phase's inputs and outputs, not the
    implementation's partial sums; kinds: fp64 (FP64 vector), mfma (FP32 matrix
    cores, with the transforms' FP32 vector work counted in), fp32 (FP32 vector).
    On the k-space route the statistics also write the data terms Y_S conj(Bhat)
    and Y_S^T conj(Ahat_S) and copy Bhat and Ahat_S, and the update adds the model
    terms (Ahat_S T_B and Bhat T_AS, T from the Grams) to form the residual's two
    gradient contractions before applying F_l^H and F_r^H."""
    P, c = n1 * n2, 8
    f1, f2 = 5 * P * math.log2(n1), 5 * P * math.log2(n2)
    a, b = n1 * r, n2 * r
    ks = 1 if kspace else 0
    return {
        "partial Grams": (c * (a + b + rows * n2) + 4 * rows + 16 * (r * r + r) + ks * 2 * c * (rows * r + b),
                          8 * (n1 + n2 + rows) * r * (r + 1) / 2 + (1 + ks) * 8 * rows * n2 * r, "fp64"),
        "ridge solve + step size": (16 * 3 * r * r + 16 * r, 8 * r ** 3 / 3 + 6 * r * r, "fp64"),
        "synthesis + row pass": (c * (P + a + b), 8 * P * r + f2, "mfma"),
        "column pass + residual": (c * (2 * P + rows * n2 + a + b) + 4 * rows, 2 * f1 + 8 * P * r, "mfma"),
        "row inverse + A grad": (c * (P + a + b), f2 + 8 * P * r, "mfma"),
        "factor updates + F_l A, F_r B": (c * 4 * (a + b) + ks * (2 * c * (rows * r + b) + 16 * 2 * r * r),
                                          (10 if kspace else 5) * a * math.log2(n1) + 8 * a
                                          + 10 * b * math.log2(n2) + 8 * b + ks * 8 * (rows + n2) * r * r, "fp32"),
        "output synthesis + row draw": (c * (P + a + b) + c * a + 4 * K, 8 * P * r + 6 * a, "mfma"),
    }


PEAK_TFS = {"fp64": 78.6, "mfma": 157.3, "fp32": 157.3}   # MI355X published: FP64 vector, FP32 matrix, FP32 vector


PHASE_KERNELS = {   # kernel of each phase in a table launch of n x n frames
    "partial Grams": "void k_lstats<",
    "ridge solve + step size": "void k_solve",
    "synthesis + row pass": "void k_synth_rowfft<{n}, FrameTable>",
    "column pass + residual": "void k_col_resid<{n}, FrameTable>",
    "row inverse + A grad": "void k_row_inv_grad<{n}, FrameTable>",
    "factor updates + F_l A, F_r B": "void k_update_ab<{n}, FrameTable>",
    "output synthesis + row draw": "void k_synth_out<",
}
COUNTERS = os.path.join(ROOT, "profiles", "step_64x256sq_r32_counters.json")


def counter_traffic(phase, n, grid=None):
    """HBM bytes per launch of the phase's kernel from the committed byte-counter
    record (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is no
    record or the kernel sources changed since it was taken."""
    try:
        with open(COUNTERS) as f:
            rec = json.load(f)
        from paper_1609_04104_amd.prof_summary import source_sha
    except (OSError, ValueError, ImportError):
        return None
    if rec.get("source_sha") != source_sha():
        return None
    want = PHASE_KERNELS[phase].format(n=n)
    hits = [v for k, v in rec.get("kernels", {}).items() if k.startswith(want) and ("FrameTable" in k or "OutTable" in k)]
    hits = [v for v in hits if v.get("dispatches", 0) > 0]
    if not hits:
        return None
    if phase == "partial Grams" and grid is not None:           # warm and informative launches differ
        hits = [v for k, v in rec["kernels"].items() if k.startswith(want) and f"[grid {grid}]" in k] or hits
    # kernels whose grid follows the sampled rows: the steady state is the smallest grid
    v = min(hits, key=lambda v: v.get("grid", 0)) if all("grid" in v for v in hits) else \
        max(hits, key=lambda v: v["dispatches"])
    return v["fetch_bytes"] + v["write_bytes"]


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else float("nan")


# ----------------------------------------------------------------------------- batched driver
class BatchDriver:
    """A fixed batch of open sequences: sequence s acquires, at frame t, rows of
    banks[s][t % len(banks[s])] (full frames on the device) -- every row for the
    first `warm` frames, then the rows its previous step drew (K[s] draws).
    Descriptor sets are built once per distinct step and replayed."""

    def __init__(self, tsl, torch, seqs, banks, Ks, warm, dev):
        self.tsl, self.seqs, self.banks, self.Ks, self.warm = tsl, seqs, banks, Ks, warm
        S = len(seqs)
        self.rows = [[torch.zeros(Ks[s], dtype=torch.int32, device=dev) for s in range(S)] for _ in range(2)]
        self.cnt = [[torch.zeros(1, dtype=torch.int32, device=dev) for _ in range(S)] for _ in range(2)]
        self.full = {q.n1: torch.arange(q.n1, dtype=torch.int32, device=dev) for q in seqs}
        self.X = [torch.empty(q.n1, q.n2, dtype=torch.complex64, device=dev) for q in seqs]
        F = 1
        for bk in banks:
            F = F * int(bk.shape[0]) // math.gcd(F, int(bk.shape[0]))
        self.period = 2 * F
        self.prepared = {}

    def frames_for(self, t):
        fr = []
        for s, q in enumerate(self.seqs):
            y = self.banks[s][t % self.banks[s].shape[0]]
            nxt = dict(K_next=self.Ks[s], rows_next=self.rows[(t + 1) % 2][s], n_next=self.cnt[(t + 1) % 2][s])
            if t < self.warm:
                fr.append(q.frame(rows=self.full[q.n1], y=y, y_full=True, X_out=self.X[s], **nxt))
            else:
                fr.append(q.frame(rows=self.rows[t % 2][s], n_rows_dev=self.cnt[t % 2][s], y=y, y_full=True,
                                  X_out=self.X[s], **nxt))
        return fr

    def key(self, t):
        return t if t < self.warm else self.warm + (t - self.warm) % self.period

    def prepare(self, t):
        k = self.key(t)
        if k not in self.prepared:
            self.prepared[k] = self.tsl.PreparedStep(self.seqs, self.frames_for(t))
        return self.prepared[k]

    def step(self, t, stream):
        self.prepare(t).launch(stream)


def time_steps(drv, warmup, steps, stream, torch, label):
    """Runs `warmup` untimed steps, times `steps` steps between two HIP events
    (nothing else enqueued in between), then runs `steps` more with an event
    after each for the per-step latency spread (not part of the throughput)."""
    for t in range(drv.warm + drv.period):          # every descriptor set built once, untimed
        drv.prepare(t)
    t = 0
    for _ in range(warmup):
        drv.step(t, stream)
        t += 1
    torch.cuda.synchronize()
    # a full collection of Python's cyclic garbage inside the loop stalls the
    # host for milliseconds; collect now and exempt everything alive from it
    gc.collect()
    gc.freeze()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    host_us = []
    w0 = time.perf_counter()
    e0.record(stream)
    for k in range(steps):
        h0 = time.perf_counter()
        drv.step(t, stream)
        host_us.append((time.perf_counter() - h0) * 1e6)
        t += 1
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = max(wall * 1e3, e0.elapsed_time(e1)) / steps
    # latency spread: the same steps with an event between consecutive ones
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        drv.step(t, stream)
        t += 1
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    slow = sorted(range(steps), key=lambda k: -step_ms[k])[:5]
    print(f"[bench] {label}: {ms_per_step:.4f} ms/step, {len(drv.seqs) * 1000.0 / ms_per_step:.0f} frames/s; "
          f"host launch us p50 {pct(host_us, 50):.1f} max {max(host_us):.1f}; evented steps p50 "
          f"{pct(step_ms, 50):.4f} ms, slowest " + ", ".join(f"#{k}: {step_ms[k]:.3f} ms" for k in slow),
          file=sys.stderr, flush=True)
    return {"ms_per_step": ms_per_step, "step_ms": step_ms, "t": t}


# ----------------------------------------------------------------------------- main
def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU; --gpus must be 1 (sharding across GPUs is "
                          "described, not built)"}))
        return 2
    import torch
    from paper_1609_04104_amd import tsl

    tsl.lib()
    torch.cuda.set_device(0)
    if a.copy_calib_mib:
        src = torch.ones(a.copy_calib_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] reference copy of {a.copy_calib_mib} MiB done", file=sys.stderr, flush=True)
        del src, dst
    S, n, r, lam, F = a.seqs, a.n, a.r, a.lam, a.frames
    K = max(1, n // 8)
    warm = 5
    print(f"[bench] generating {S} x {F} frames of {n}x{n}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    data = make_inputs(S, n, r, F, a.procs)
    print(f"[bench] inputs in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    Kd = [torch.from_numpy(d[0]).to(dev) for d in data]                  # [F, n, n] per sequence
    full = torch.arange(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def open_seq(s, route=a.route):
        A0, B0 = data[s][1], data[s][2]
        return tsl.Sequence(n, n, r, lam, torch.from_numpy(A0).to(dev), torch.from_numpy(B0).to(dev),
                            seed=1609, stream_id=s, route=route)

    # ------------------------------------------------------------------ batched
    seqs = [open_seq(s) for s in range(S)]
    drv = BatchDriver(tsl, torch, seqs, Kd, [K] * S, warm, dev)
    res = time_steps(drv, a.warmup, a.steps, stream, torch, "batched")
    ms_per_step, step_ms, t = res["ms_per_step"], res["step_ms"], res["t"]
    value = S * 1000.0 / ms_per_step
    bad = [q for q in seqs if q.status() != 0]
    frames_for, cnt = drv.frames_for, drv.cnt

    # per-phase split (profiling form of the same step, HIP events between phases)
    phase_ms = [0.0] * tsl.N_PHASES
    for _ in range(a.phase_steps):
        phase_ms = tsl.step_many_timed(seqs, frames_for(t), phase_ms, stream)
        t += 1
    phase_ms = [x / a.phase_steps for x in phase_ms]
    mean_rows = float(np.mean([int(cnt[t % 2][i].item()) for i in range(S)]))
    work = phase_work(n, n, r, mean_rows, K, kspace=a.route == "kspace")
    dom = int(np.argmax(phase_ms))
    dname = tsl.PHASES[dom]
    dbytes, dflops, kind = work[dname]
    dbytes, dflops = dbytes * S, dflops * S
    dt = phase_ms[dom] * 1e-3
    ai = dflops / dbytes
    ridge = PEAK_TFS[kind] * 1e12 / (HBM_PEAK_GBS * 1e9)
    if ai > ridge:
        roof = {"bound": "mfma" if kind == "mfma" else "alu", "achieved": dflops / dt / 1e12,
                "peak": PEAK_TFS[kind], "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": dbytes / dt / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    gx = (-(-n // 64)) * 2 + (-(-K // 32)) * (1 + (-(-n // 32)))    # statistics blocks per frame
    roof["traffic"] = counter_traffic(dname, n, grid=gx * 256 * (-(-S // 8) * 8))
    roof["kernel"] = dname
    roof["algorithmic_bytes_per_launch"] = dbytes
    roof["algorithmic_flops_per_launch"] = dflops
    roof["avg_launch_ms"] = phase_ms[dom]
    for q in seqs:
        q.close()

    # ------------------------------------------------------------------ the same batch on the other route
    other = "frame" if a.route == "kspace" else "kspace"
    other_leg = None
    if a.frame_route_steps > 0:
        oseqs = [open_seq(s, other) for s in range(S)]
        odrv = BatchDriver(tsl, torch, oseqs, Kd, [K] * S, warm, dev)
        ores = time_steps(odrv, a.warmup, a.frame_route_steps, stream, torch, f"{other} route")
        ophase = [0.0] * tsl.N_PHASES
        ot = ores["t"]
        for _ in range(a.phase_steps):
            ophase = tsl.step_many_timed(oseqs, odrv.frames_for(ot), ophase, stream)
            ot += 1
        other_leg = {"route": other, "frames_per_s": S * 1000.0 / ores["ms_per_step"],
                     "ms_per_step": ores["ms_per_step"],
                     "phases_ms": {name: ophase[i] / a.phase_steps for i, name in enumerate(tsl.PHASES)}}
        if other == "frame":
            other_leg["roofline_passes"] = frame_pass_rooflines(
                other_leg["phases_ms"], phase_ms, n, r, mean_rows, K, S, "frame-route passes, 64-sequence batch")
        bad += [q for q in oseqs if q.status() != 0]
        for q in oseqs:
            q.close()
        print(f"[bench] {other} route {other_leg['frames_per_s']:.0f} frames/s", file=sys.stderr, flush=True)

    # ------------------------------------------------------------------ beyond the Infinity Cache
    mall = None if a.mall_seqs <= 0 else mall_leg(a, tsl, torch, dev, stream, n, r, lam, K, warm)

    # ------------------------------------------------------------------ plain
    q = open_seq(0)
    pr = [torch.zeros(K, dtype=torch.int32, device=dev) for _ in range(2)]
    pc = [torch.zeros(1, dtype=torch.int32, device=dev) for _ in range(2)]
    X0 = torch.empty(n, n, dtype=torch.complex64, device=dev)

    def plain_frame(t):
        nxt = dict(K_next=K, rows_next=pr[(t + 1) % 2], n_next=pc[(t + 1) % 2])
        if t < warm:
            return q.frame(rows=full, y=Kd[0][t % F], y_full=True, X_out=X0, **nxt)
        return q.frame(rows=pr[t % 2], n_rows_dev=pc[t % 2], y=Kd[0][t % F], y_full=True, X_out=X0, **nxt)

    period = 2 * F
    pframes = [plain_frame(t) for t in range(warm + period)]

    def pf(t):
        return pframes[t if t < warm else warm + (t - warm) % period]

    for t in range(a.warmup):
        q.push(pf(t), stream)
    torch.cuda.synchronize()
    P = a.plain_frames
    pev = [torch.cuda.Event(enable_timing=True) for _ in range(P + 1)]
    gc.collect()
    gc.freeze()
    w0 = time.perf_counter()
    pev[0].record(stream)
    for k in range(P):
        q.push(pf(a.warmup + k), stream)
        pev[k + 1].record(stream)
    torch.cuda.synchronize()
    pwall = time.perf_counter() - w0
    plain_ms = [pev[k].elapsed_time(pev[k + 1]) for k in range(P)]
    plain_fps = P / max(pwall, pev[0].elapsed_time(pev[-1]) * 1e-3)
    bad += [q] if q.status() != 0 else []
    q.close()
    print(f"[bench] plain {plain_fps:.0f} frames/s", file=sys.stderr, flush=True)

    # ------------------------------------------------------------------ mixed shapes, served arrivals
    mixed = None if a.no_mixed else mixed_leg(a, tsl, torch, dev, stream)
    served = None if a.no_serve else serving_leg(a, tsl, torch, dev, stream)

    # ------------------------------------------------------------------ parity + CPU oracle
    parity, cpu = None, None
    if not a.no_cpu:
        parity, cpu = oracle_leg(a, data, Kd, n, r, lam, K, warm, dev, tsl, torch)

    out = {
        "metric": "frames/s at 256²,R=32 (batched vs plain); p50/p99 frame latency",
        "value": value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": f"{S} concurrent {n}x{n} cine sequences, R={r}, lambda={lam}, informative row "
                        f"sampling with K={K} draws (12.5% line budget) after 5 fully sampled frames; one step "
                        f"= one frame of every sequence through the whole step incl. the next-row draw",
            "sequences": S, "n1": n, "n2": n, "r": r, "lambda": lam, "K": K,
            "precision": "complex FP32 frame path, FP64 RxR statistics and solve",
            "line_route": a.route,
        },
        "latency_ms": {"batched_p50": pct(step_ms, 50), "batched_p99": pct(step_ms, 99),
                       "plain_p50": pct(plain_ms, 50), "plain_p99": pct(plain_ms, 99),
                       **({"served_p50": served["loads"][0]["batched"]["latency_p50_ms"],
                           "served_p99": served["loads"][0]["batched"]["latency_p99_ms"],
                           "served_plain_p50": served["loads"][0]["plain"]["latency_p50_ms"],
                           "served_plain_p99": served["loads"][0]["plain"]["latency_p99_ms"]}
                          if served else {})},
        "plain": {"frames_per_s": plain_fps, "ms_per_frame": 1e3 / plain_fps},
        "route": a.route,
        "other_route": other_leg,
        "mixed": mixed,
        "beyond_mall": mall,
        "serving": served,
        "batched_over_plain": value / plain_fps,
        "phases_ms": {name: phase_ms[i] for i, name in enumerate(tsl.PHASES)},
        "tuned_output_tile": {"batched": tsl.output_tile(n, n, r, S), "plain": tsl.output_tile(n, n, r, 1)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "device_status_errors": len(bad),
    }
    print(json.dumps(out))
    return 0


def frame_pass_rooflines(phases, kspace_phases, n, r, rows, K, S, label):
    """HBM rooflines of the frame route's three frame-sized passes from their
    event-bracketed phase times.  A bracket adds a fixed overhead (the events
    and the launch gap), measured on a phase that launches nothing in the same
    run (the synthesis + row pass of the k-space route) and subtracted."""
    overhead = kspace_phases.get("synthesis + row pass", 0.0) if isinstance(kspace_phases, dict) else \
        kspace_phases[2]
    work = phase_work(n, n, r, rows, K, kspace=False)
    out = {"label": label, "bracket_overhead_ms": overhead, "passes": {}}
    for name in ("synthesis + row pass", "column pass + residual", "row inverse + A grad"):
        ms = phases[name]
        net = max(ms - overhead, 1e-6)
        b, fl = work[name][0] * S, work[name][1] * S
        hbm = b / (net * 1e-3) / 1e9 / HBM_PEAK_GBS
        mfma = fl / (net * 1e-3) / 1e12 / PEAK_TFS["mfma"]
        out["passes"][name] = {"algorithmic_bytes_per_launch": b, "algorithmic_flops_per_launch": fl,
                               "bracketed_ms": ms, "net_ms": net,
                               "achieved_GBps": b / (net * 1e-3) / 1e9, "frac_of_hbm": hbm,
                               "achieved_TFLOPs": fl / (net * 1e-3) / 1e12, "frac_of_fp32_matrix": mfma,
                               "bound": "hbm" if hbm >= mfma else "mfma"}
    return out


def mall_leg(a, tsl, torch, dev, stream, n, r, lam, K, warm):
    """Both routes on a batch whose frame-sized arrays exceed the 256 MB
    Infinity Cache (1024 x 256^2: 512 MiB per frame array), so the frame
    route's passes stream from HBM.  Inputs are CN(0, 1) k-space frames made on
    the device (two per sequence, cycled): the work of a step does not depend
    on their content."""
    S = a.mall_seqs
    g = torch.Generator(device=dev)
    g.manual_seed(1609)
    banks = [torch.randn(2, n, n, dtype=torch.complex64, device=dev, generator=g) for _ in range(S)]
    out = {"workload": f"{S} sequences of {n}x{n}, R={r}, informative rows (K={K}) after {warm} full frames; "
                       f"synthetic CN(0,1) k-space frames", "sequences": S}
    for route in ("kspace", "frame"):
        seqs = []
        for s in range(S):
            A0 = (torch.randn(n, r, dtype=torch.complex64, device=dev, generator=g) / math.sqrt(n)).contiguous()
            B0 = (torch.randn(n, r, dtype=torch.complex64, device=dev, generator=g) / math.sqrt(n)).contiguous()
            seqs.append(tsl.Sequence(n, n, r, lam, A0, B0, seed=7, stream_id=s, route=route))
        drv = BatchDriver(tsl, torch, seqs, banks, [K] * S, warm, dev)
        res = time_steps(drv, warm + 2, a.mall_steps, stream, torch, f"beyond-MALL {route}")
        ph = [0.0] * tsl.N_PHASES
        t = res["t"]
        for _ in range(3):
            ph = tsl.step_many_timed(seqs, drv.frames_for(t), ph, stream)
            t += 1
        leg = {"frames_per_s": S * 1000.0 / res["ms_per_step"], "ms_per_step": res["ms_per_step"],
               "phases_ms": {name: ph[i] / 3 for i, name in enumerate(tsl.PHASES)},
               "device_status_errors": sum(1 for q in seqs if q.status() != 0)}
        out[route] = leg
        for q in seqs:
            q.close()
        drv.prepared.clear()
        torch.cuda.synchronize()
    out["frame"]["roofline_passes"] = frame_pass_rooflines(out["frame"]["phases_ms"], out["kspace"]["phases_ms"],
                                                           n, r, K, K, S, f"frame-route passes, {S}-sequence batch")
    return out


def mixed_leg(a, tsl, torch, dev, stream):
    """64 concurrent sequences of mixed shapes (128x128, 192x160, 256x256), ranks
    16/32/64 and accelerations 4-12 (K = N1/acceleration draws), one step per frame."""
    from paper_1609_04104_amd import inputs as I
    specs = I.mixed_batch_specs(64)
    shapes = sorted({(d["n1"], d["n2"]) for d in specs})
    banks = {sh: torch.from_numpy(I.phantom_bank(sh[0], a.bank_frames, seq=k, n2=sh[1], config=4)).to(dev)
             for k, sh in enumerate(shapes)}
    seqs = []
    for d in specs:
        A0, B0 = I.init_factors(d["n1"], d["n2"], d["r"], I.rng_for(4, d["seq"], 3))
        seqs.append(tsl.Sequence(d["n1"], d["n2"], d["r"], a.lam, torch.from_numpy(A0).to(dev),
                                 torch.from_numpy(B0).to(dev), seed=1609, stream_id=1000 + d["seq"]))
    Ks = [max(1, round(d["n1"] / d["accel"])) for d in specs]
    drv = BatchDriver(tsl, torch, seqs, [banks[(d["n1"], d["n2"])] for d in specs], Ks, 5, dev)
    res = time_steps(drv, a.warmup, a.mixed_steps, stream, torch, "mixed")
    bad = sum(1 for q in seqs if q.status() != 0)
    for q in seqs:
        q.close()
    n_pix = sum(d["n1"] * d["n2"] for d in specs)
    return {
        "workload": "64 sequences: 22 x 128x128, 21 x 192x160, 21 x 256x256 (seeded order), R in {16, 32, 64}, "
                    "acceleration 4-12, informative rows after 5 full frames, lambda 0.05",
        "frames_per_s": len(seqs) * 1000.0 / res["ms_per_step"],
        "ms_per_step": res["ms_per_step"],
        "step_p50_ms": pct(res["step_ms"], 50), "step_p99_ms": pct(res["step_ms"], 99),
        "pixels_per_step": n_pix, "device_status_errors": bad,
    }


def serving_leg(a, tsl, torch, dev, stream):
    """Scans arriving as a Poisson process, each streaming frames, served by
    continuous batching and by the plain one-frame-at-a-time loop."""
    from paper_1609_04104_amd import inputs as I
    from paper_1609_04104_amd import serve as SV
    specs = I.serving_specs(a.serve_scans, a.serve_rate)
    sizes = sorted({d["n"] for d in specs})
    banks = {n: torch.from_numpy(I.phantom_bank(n, a.bank_frames, seq=k)).to(dev) for k, n in enumerate(sizes)}
    init = {d["scan"]: (torch.from_numpy(d["A0"]).to(dev), torch.from_numpy(d["B0"]).to(dev)) for d in specs}
    free, _ = torch.cuda.mem_get_info()
    budget = free // 2
    loads = [float(x) for x in a.serve_loads.split(",") if x]
    last_arrival = max(d["arrival"] for d in specs)
    out = []
    for k in loads:
        fps = 30.0 * k
        row = {"load": k, "frame_rate_per_scan": fps,
               "offered_frames_per_s": len(specs) * a.serve_T / (last_arrival / k + a.serve_T / fps)}
        for mode in ("batched", "plain"):
            scans = [SV.Scan(d["scan"], d["n"], d["r"], a.lam, *init[d["scan"]], banks[d["n"]], a.serve_T,
                             d["arrival"] / k, fps) for d in specs]
            gc.collect()
            r = SV.serve(scans, budget, stream, plain=(mode == "plain"), time_limit=a.serve_limit)
            row[mode] = r
            print(f"[bench] served load x{k:g} {mode}: {r['frames']} frames, {r['frames_per_s']:.0f} frames/s, "
                  f"latency p50 {r['latency_p50_ms']:.2f} ms p99 {r['latency_p99_ms']:.2f} ms, "
                  f"mean batch {r['mean_batch']:.1f}", file=sys.stderr, flush=True)
        out.append(row)
    return {
        "workload": f"{a.serve_scans} scans, Poisson arrivals at {a.serve_rate:g}/s x load, N x N with N in "
                    f"{sizes}, R in {{16, 32, 48, 64}}, {a.serve_T} frames each at 30/s x load, informative rows "
                    f"(K = N/8) after 5 full frames; HBM pool budget {budget} bytes",
        "loads": out,
    }


def oracle_leg(a, data, Kd, n, r, lam, K, warm, dev, tsl, torch):
    """FP64 oracle on sequence 0: teacher-forced parity of the GPU's plain path,
    then the oracle's own frames/s on a bounded sample of the same workload."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    kspace, A0, B0 = data[0]
    F = kspace.shape[0]
    # parity: GPU plain path draws its own rows; the oracle follows them
    q = tsl.Sequence(n, n, r, lam, torch.from_numpy(A0).to(dev), torch.from_numpy(B0).to(dev),
                     seed=1609, stream_id=0)
    o = oracle.TslOracle(n, n, r, lam, A0, B0)
    full = torch.arange(n, dtype=torch.int32, device=dev)
    rows_d = torch.zeros(K, dtype=torch.int32, device=dev)
    cnt_d = torch.zeros(1, dtype=torch.int32, device=dev)
    X = torch.empty(n, n, dtype=torch.complex64, device=dev)
    Ah = torch.empty(n, r, dtype=torch.complex64, device=dev)
    rows_h = np.arange(n, dtype=np.int32)
    worst, agree, draws = 0.0, 0, 0
    n_par = 20
    for t in range(n_par):
        rin = full if t < warm else torch.from_numpy(rows_h).to(dev)
        fr = q.frame(rows=rin, y=Kd[0][t % F], y_full=True, X_out=X, K_next=K, rows_next=rows_d, n_next=cnt_d)
        q.push(fr)
        torch.cuda.synchronize()
        s = o.push_lines(rows_h, kspace[t % F][rows_h])
        worst = max(worst, float(np.linalg.norm(X.cpu().numpy() - s.X) / np.linalg.norm(s.X)))
        q.factors(Ahat=Ah)
        nr = int(cnt_d.item())
        g_rows = rows_d.cpu().numpy()[:nr].copy()
        o_rows, _ = oracle.draw_lines(Ah.cpu().numpy(), n, K, 1609, 0, t + 2)
        draws += 1
        agree += int(np.array_equal(o_rows, g_rows))
        rows_h = g_rows if t + 1 >= warm else np.arange(n, dtype=np.int32)
    q.close()
    parity = {"frames": n_par, "max_nrmse_X_vs_oracle": worst,
              "row_draws_bit_exact": f"{agree}/{draws}", "tolerance": 1e-4}
    # CPU baseline: the oracle alone (its own FP64 draws), bounded time, with
    # the BLAS threads it gets by default and again with one thread
    def oracle_rate(seconds):
        o = oracle.TslOracle(n, n, r, lam, A0, B0)
        rows_o = np.arange(n, dtype=np.int32)
        frames = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            o.push_lines(rows_o, kspace[frames % F][rows_o])
            Ah_o, _ = o.kspace_factors()
            frames += 1
            rows_o = (oracle.draw_lines(Ah_o, n, K, 1609, 0, frames + 1)[0] if frames >= warm
                      else np.arange(n, dtype=np.int32))
        return frames, time.perf_counter() - t0

    frames, el = oracle_rate(a.cpu_seconds)
    f1, el1 = None, None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            f1, el1 = oracle_rate(a.cpu_seconds / 2)
    except Exception:
        pass
    host = {"nproc": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count(),
            "cpu": cpu_model()}
    cpu = {"value": frames / el, "unit": "frames/s", "cores": threads, "kind": "oracle",
           "sample": f"{frames} frames of sequence 0 ({n}x{n}, R={r}, informative rows) in {el:.1f}s, "
                     f"FP64 NumPy with dense DFT matrices, {threads} BLAS threads",
           "value_1thread": (f1 / el1) if f1 else None,
           "sample_1thread": (f"{f1} frames in {el1:.1f}s with one BLAS thread" if f1 else None),
           "host": host}
    print(f"[bench] oracle {cpu['value']:.1f} frames/s on {threads} threads"
          f"{'' if not f1 else f', {f1 / el1:.1f} on one'}; parity {parity}", file=sys.stderr, flush=True)
    return parity, cpu


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    sys.exit(main())
