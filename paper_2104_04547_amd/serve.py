"""Serving: a thin wrapper over the engine entry points and an open-loop load generator.

The engine (cf_engine_* in libcf.so) does the batching, scheduling, hipGraph replay
and latency stamping natively; this module only submits requests on a Poisson
clock, polls tickets and summarises the latencies the engine reports.
"""
from __future__ import annotations

import threading
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import cfabi


class Engine:
    def __init__(self, arch, params, precision: str = "bf16", n_slots: int = 4, slot_poses: int = 512,
                 slot_atoms: int = 512 * 1600, hbm_budget_bytes: int = 64 << 30, use_graphs: bool = True):
        prec = {"bf16": cfabi.CF_PREC_BF16, "fp32": cfabi.CF_PREC_FP32}[precision]
        self.h = cfabi.cf_engine_create(cfabi.pack_model(arch, params), prec, n_slots, slot_poses, slot_atoms,
                                        hbm_budget_bytes, use_graphs)
        self.slot_poses = slot_poses

    def submit(self, batch, G: int) -> int:
        return cfabi.cf_engine_submit(self.h, batch.atom_off, batch.xyz, batch.feat, batch.is_lig, G)

    def poll(self, ticket: int, n_poses: int):
        return cfabi.cf_engine_poll(self.h, ticket, n_poses)

    def result(self, ticket: int, n_poses: int, timeout_s: float = 120.0):
        t0 = time.perf_counter()
        while True:
            done, scores, lat = self.poll(ticket, n_poses)
            if done:
                return scores, lat
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError("engine request did not finish")
            time.sleep(0.0005)

    def cancel(self, ticket: int) -> bool:
        return cfabi.cf_engine_cancel(self.h, ticket)

    def wait_all(self):
        cfabi.cf_engine_wait_all(self.h)

    def info(self):
        return cfabi.cf_engine_info(self.h)

    def close(self):
        if self.h:
            cfabi.cf_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Span:
    """Poses [start, start + k) of a pose pool as a request batch: views of the
    pool's arrays (the pool holds max_poses - 1 poses past its cyclic end, so every
    span is contiguous) and offsets rebased to 0.  Built when the request is
    submitted, so a long stream holds no per-request copies."""

    def __init__(self, pool, start: int, k: int):
        a, b = int(pool.atom_off[start]), int(pool.atom_off[start + k])
        self.atom_off = np.ascontiguousarray(pool.atom_off[start:start + k + 1] - pool.atom_off[start])
        self.xyz, self.feat, self.is_lig = pool.xyz[a:b], pool.feat[a:b], pool.is_lig[a:b]
        self.n_poses = k

    @property
    def n_atoms(self) -> int:
        return int(self.atom_off[-1])


class Requests:
    """n requests of U{1..max_poses} consecutive poses (cycling through the first
    `period` poses of the pool), each with a grid size drawn uniformly from `grids`;
    request i is materialised as views of the pool when it is read."""

    def __init__(self, pool, n_requests: int, rng: np.random.Generator, max_poses: int = 256,
                 grids: Sequence[int] = (48, 64)):
        self.pool = pool
        self.period = pool.n_poses - (max_poses - 1)
        assert self.period >= 1, "pool needs max_poses - 1 poses past its period"
        self.k = rng.integers(1, max_poses + 1, size=n_requests)
        self.G = rng.choice(np.asarray(grids), size=n_requests)
        starts = np.concatenate([[0], np.cumsum(self.k)[:-1]])
        self.start = starts % self.period

    def __len__(self):
        return len(self.k)

    def __getitem__(self, i):
        return _Span(self.pool, int(self.start[i]), int(self.k[i])), int(self.G[i])

    def __iter__(self):
        for i in range(len(self)):
            yield self[i]

    @property
    def total_poses(self) -> int:
        return int(self.k.sum())


def make_requests(pool, n_requests: int, rng: np.random.Generator, max_poses: int = 256,
                  grids: Sequence[int] = (48, 64)):
    """Requests of U{1..max_poses} consecutive poses from a pose pool, each with a
    grid size drawn uniformly from `grids` (see Requests)."""
    return Requests(pool, n_requests, rng, max_poses, grids)


def warm_up(engine: Engine, pool, grids: Sequence[int] = (48, 64), n_slots: int = 4):
    """Score one batch per (grid, bucket, slot), twice, so that every hipGraph is
    captured before timing: the first pass grows each slot's scratch to its final
    size (which drops the graphs captured against smaller buffers), the second
    captures the graphs that replay from then on."""
    buckets = []
    b = 16
    while b <= engine.slot_poses:
        buckets.append(b)
        b *= 2
    for _ in range(2):
        tickets = []
        for _ in range(n_slots):
            for G in grids:
                for b in buckets:
                    n = min(b, 256)
                    sub = pool.select(list(range(n)))
                    tickets.append((engine.submit(sub, G), n))
        for t, n in tickets:
            engine.result(t, n)


def run_open_loop(engine: Engine, requests, rate_rps: float, seed: int = 0) -> Dict:
    """Submit requests at Poisson arrival times (open loop) and collect latencies."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_rps, size=len(requests))
    progress_s = 30.0
    pending = {}
    lock = threading.Lock()
    lat: List[float] = []
    done_poses = [0]
    finished = threading.Event()

    def sender():
        t_next = time.perf_counter()
        for (b, G), gap in zip(requests, gaps):
            t_next += gap
            dt = t_next - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            t = engine.submit(b, G)
            with lock:
                pending[t] = b.n_poses
        finished.set()

    t0 = time.perf_counter()
    t_report = t0 + progress_s
    th = threading.Thread(target=sender, daemon=True)
    th.start()
    while True:
        if time.perf_counter() > t_report:
            t_report += progress_s
            print(f"[serve] {len(lat)} requests, {done_poses[0]} poses done after "
                  f"{time.perf_counter() - t0:.0f} s", flush=True)
        with lock:
            items = list(pending.items())
        for t, n in items:
            ok, _, l = engine.poll(t, n)
            if ok:
                lat.append(l)
                done_poses[0] += n
                with lock:
                    del pending[t]
        if finished.is_set():
            with lock:
                if not pending:
                    break
        time.sleep(0.0005)
    t1 = time.perf_counter()
    th.join()
    lat_a = np.array(lat)
    return dict(requests=len(lat), poses=done_poses[0], seconds=t1 - t0, poses_per_s=done_poses[0] / (t1 - t0),
                offered_rps=rate_rps, p50_ms=float(np.percentile(lat_a, 50)), p99_ms=float(np.percentile(lat_a, 99)),
                mean_ms=float(lat_a.mean()), max_ms=float(lat_a.max()))
