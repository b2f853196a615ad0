"""Streaming AS-TAX serving with continuous batching on one GPU.

Frame requests arrive over time from arrays of different sizes, sampling rates
and record lengths.  The server keeps one plan per array set-up resident on the
device (kz tables, basis, twiddles: the propagator inputs), and runs a single
scheduler loop that

  * moves arrived requests into per-(plan, record length) queues,
  * polls in-flight batches for completion (HIP events), releasing their HBM
    and their stream slot and recording each request's latency,
  * admits new batches while a stream slot is free and the batch's device
    memory (RF, workspace, outputs) fits the remaining HBM budget: the oldest
    waiting request picks the queue, and the batch takes up to `max_batch`
    requests of that queue, shrinking until it fits.

A batch is one pam_as_tax call (one plan, one record length); batches of
different arrays run concurrently on separate streams, so requests that arrive
while others are on the GPU join as soon as a slot and memory free up.  Every
request's RF is copied host->device on its batch's stream and its image comes
back device->host on the same stream before completion is signalled.
"""
from __future__ import annotations

import argparse
import collections
import json
import sys
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import pam, synth


@dataclass(frozen=True)
class ArrayKey:
    """Set-up that selects a plan: element count and sampling rate (pitch and grid follow)."""
    n_elements: int
    fs_hz: float


@dataclass
class Request:
    rid: int
    key: ArrayKey
    n_t: int
    rf: object                    # pinned host tensor [L][n_t] float32
    t_arrival: float = 0.0        # seconds from the start of the run
    t_done: Optional[float] = None
    image: Optional[np.ndarray] = None
    status: str = "pending"


@dataclass
class _Batch:
    reqs: List[Request]
    stream_slot: int
    event: object
    mem: int
    keep: list = field(default_factory=list)
    image_host: object = None


class Server:
    def __init__(self, device: int = 0, hbm_budget: int = 16 << 30, max_batch: int = 16,
                 n_streams: int = 4, precision: str = "fp32", max_samples: int = 16384):
        import torch
        self.torch = torch
        self.device = torch.device(f"cuda:{device}")
        self.dev_index = device
        self.hbm_budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.precision = precision
        self.max_samples = int(max_samples)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.free_slots = list(range(n_streams))
        self.plans: Dict[ArrayKey, pam.Plan] = {}
        self.queues: Dict[Tuple[ArrayKey, int], collections.deque] = collections.defaultdict(collections.deque)
        self.inflight: List[_Batch] = []
        self.mem_in_use = 0
        self.stats = collections.Counter()
        self.batch_sizes: List[int] = []

    # -- plans -------------------------------------------------------------------
    def geometry(self, key: ArrayKey):
        return synth.cfg5_geometry(key.n_elements, key.fs_hz, self.max_samples)

    def plan(self, key: ArrayKey) -> pam.Plan:
        p = self.plans.get(key)
        if p is None:
            p = pam.pam_plan(self.geometry(key), self.dev_index, self.precision)
            self.plans[key] = p
        return p

    def close(self):
        self.drain()
        for p in self.plans.values():
            pam.pam_destroy(p)
        self.plans.clear()

    # -- memory ------------------------------------------------------------------
    def batch_bytes(self, key: ArrayKey, n_t: int, n: int) -> int:
        p = self.plan(key)
        ws = pam.pam_workspace_size(p, n, n_t)
        rf = n * key.n_elements * n_t * 4
        img = n * p.n_z * p.n_x * 4
        return ws + rf + img

    # -- scheduling ----------------------------------------------------------------
    def submit(self, req: Request):
        self.plan(req.key)
        self.queues[(req.key, req.n_t)].append(req)

    def _poll(self, now: float):
        done = [b for b in self.inflight if b.event.query()]
        for b in done:
            self.inflight.remove(b)
            imgs = b.image_host.numpy()
            for i, r in enumerate(b.reqs):
                r.image = imgs[i].copy()
                r.t_done = now
                r.status = "done"
            self.mem_in_use -= b.mem
            self.free_slots.append(b.stream_slot)
            self.stats["completed"] += len(b.reqs)
        return len(done)

    def _launch(self, key: ArrayKey, n_t: int, reqs: List[Request], mem: int):
        torch = self.torch
        slot = self.free_slots.pop()
        stream = self.streams[slot]
        p = self.plan(key)
        n = len(reqs)
        with torch.cuda.stream(stream):
            rf = torch.empty((n, key.n_elements, n_t), dtype=torch.float32, device=self.device)
            for i, r in enumerate(reqs):
                rf[i].copy_(r.rf, non_blocking=True)
            image = torch.empty((n, p.n_z, p.n_x), dtype=torch.float32, device=self.device)
            ws = torch.empty(pam.pam_workspace_size(p, n, n_t), dtype=torch.uint8, device=self.device)
            pam.pam_as_tax(p, rf, image, None, None, ws, stream, n_t)
            image_host = torch.empty(image.shape, dtype=torch.float32, pin_memory=True)
            image_host.copy_(image, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.mem_in_use += mem
        self.inflight.append(_Batch(reqs, slot, ev, mem, keep=[rf, image, ws], image_host=image_host))
        self.batch_sizes.append(n)
        self.stats["batches"] += 1
        self.stats["max_inflight"] = max(self.stats["max_inflight"], len(self.inflight))

    def _admit(self) -> int:
        launched = 0
        while self.free_slots:
            heads = [(q[0].t_arrival, k) for k, q in self.queues.items() if q]
            if not heads:
                break
            _, (key, n_t) = min(heads, key=lambda h: h[0])
            q = self.queues[(key, n_t)]
            n = min(self.max_batch, len(q))
            free = self.hbm_budget - self.mem_in_use
            while n > 0 and self.batch_bytes(key, n_t, n) > free:
                n -= 1
            if n == 0:
                if not self.inflight:
                    # even one frame exceeds the whole budget: refuse it rather than wait forever
                    r = q.popleft()
                    r.status = "rejected"
                    self.stats["rejected"] += 1
                    continue
                self.stats["admission_stalls"] += 1
                break
            reqs = [q.popleft() for _ in range(n)]
            self._launch(key, n_t, reqs, self.batch_bytes(key, n_t, n))
            launched += 1
        return launched

    def drain(self):
        while self.inflight:
            self.torch.cuda.synchronize(self.device)
            self._poll(time.perf_counter())

    def run(self, requests: List[Request], realtime: bool = True,
            deadline_s: Optional[float] = None) -> List[Request]:
        """Serve requests whose t_arrival are offsets (s) from now; returns them with latencies.

        With a deadline, no batch is admitted after deadline_s: requests still queued or not
        yet arrived are marked "unserved" and only the batches in flight are drained."""
        order = sorted(requests, key=lambda r: r.t_arrival)
        for r in order:
            self.plan(r.key)          # plans exist before the clock starts (pre-run)
        pending = collections.deque(order)
        t0 = time.perf_counter()
        while pending or self.inflight or any(self.queues.values()):
            now = time.perf_counter() - t0
            if deadline_s is not None and now > deadline_s:
                for r in list(pending) + [r for q in self.queues.values() for r in q]:
                    r.status = "unserved"
                    self.stats["unserved"] += 1
                pending.clear()
                for q in self.queues.values():
                    q.clear()
                while self.inflight:
                    self.torch.cuda.synchronize(self.device)
                    self._poll(time.perf_counter() - t0)
                break
            while pending and (pending[0].t_arrival <= now or not realtime):
                self.submit(pending.popleft())
            polled = self._poll(now)
            launched = self._admit()
            if not polled and not launched:
                nxt = pending[0].t_arrival - now if pending else 1e-4
                time.sleep(min(max(nxt, 0.0), 2e-4))
        return order


# ----------------------------------------------------------------------------
# Load generation
# ----------------------------------------------------------------------------

ARRAYS = (64, 128, 256)
RATES = (20e6, 40e6)
LENGTHS = (1024, 2048, 4096, 8192, 16384)


def make_pool(seed: int = 0, arrays=ARRAYS, rates=RATES, lengths=LENGTHS):
    """One synthetic frame per (array, fs, record length) as pinned host tensors."""
    import torch
    pool = {}
    rng = np.random.default_rng(seed)
    for L in arrays:
        for fs in rates:
            g = synth.cfg5_geometry(L, fs, max(lengths))
            half = L * g.pitch_m / 2 / synth.MM
            for n_t in lengths:
                em = synth._random_emitters(rng, int(rng.integers(1, 6)), (-0.8 * half, 0.8 * half), (20, 60), [])
                rf = synth.render(g, em, rng, n_t=n_t, snr_db=20.0)
                pool[(ArrayKey(L, fs), n_t)] = torch.from_numpy(rf).pin_memory()
    return pool


def poisson_requests(pool, rate_hz: float, n: int, seed: int = 1) -> List[Request]:
    rng = np.random.default_rng(seed)
    keys = list(pool.keys())
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        key, n_t = keys[int(rng.integers(0, len(keys)))]
        out.append(Request(i, key, n_t, pool[(key, n_t)], t_arrival=t))
    return out


def summarize(reqs: List[Request], rate_hz: float) -> dict:
    done = [r for r in reqs if r.status == "done"]
    lat = np.array([1e3 * (r.t_done - r.t_arrival) for r in done]) if done else np.zeros(1)
    span = (max(r.t_done for r in done) - min(r.t_arrival for r in reqs)) if done else 0.0
    return {"offered_fps": rate_hz, "requests": len(reqs), "completed": len(done),
            "rejected": sum(r.status == "rejected" for r in reqs),
            "unserved": sum(r.status == "unserved" for r in reqs),
            "completed_fps": round(len(done) / span, 2) if span > 0 else None,
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3)}


def main(argv=None):
    ap = argparse.ArgumentParser(description="Poisson load test of the continuous-batching server")
    ap.add_argument("--loads", default="100,1000,5000")
    ap.add_argument("--requests", type=int, default=300, help="requests per offered load")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--max-batch", type=int, default=16)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--hbm-gib", type=float, default=32.0)
    ap.add_argument("--max-samples", type=int, default=16384)
    args = ap.parse_args(argv)
    lengths = tuple(n for n in LENGTHS if n <= args.max_samples)
    t = time.perf_counter()
    pool = make_pool(lengths=lengths)
    print(f"pool of {len(pool)} frames in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    out = {"precision": args.precision, "max_batch": args.max_batch, "streams": args.streams,
           "hbm_budget_gib": args.hbm_gib, "mix": "64/128/256 elements x 20/40 MHz x record lengths "
           + "/".join(map(str, lengths)), "loads": []}
    srv = Server(max_batch=args.max_batch, n_streams=args.streams, precision=args.precision,
                 hbm_budget=int(args.hbm_gib * (1 << 30)), max_samples=args.max_samples)
    try:
        warm = poisson_requests(pool, 1e6, len(pool), seed=99)
        srv.run(warm, realtime=False)
        for rate in [float(x) for x in args.loads.split(",") if x]:
            srv.batch_sizes.clear()
            reqs = poisson_requests(pool, rate, args.requests, seed=int(rate))
            srv.run(reqs)
            s = summarize(reqs, rate)
            s["mean_batch"] = round(float(np.mean(srv.batch_sizes)), 2) if srv.batch_sizes else 0
            s["admission_stalls"] = srv.stats["admission_stalls"]
            out["loads"].append(s)
            print(json.dumps(s), file=sys.stderr, flush=True)
    finally:
        srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
