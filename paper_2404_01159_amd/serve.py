"""Serving loop: independent RVEA runs arriving over time, continuously batched.

Requests (problem, m, d, N, K, seed, generations) arrive at given times.  A
request is admitted, in arrival order, once a batch slot is free and its
workspace (rvea_footprint bytes) fits in the device arena; its population,
reference vectors and generation counter then stay resident in its slice of
the arena.  Every tick advances every admitted run by one generation with one
rvea_batch_step (one launch per phase, replayed as a graph while membership
is stable); runs that have done their generations leave the batch at the tick
boundary and free their memory, and queued requests take their place.
Latency is arrival to completion of the last generation.  Once no request
is waiting, the ticks up to the next completion are enqueued together.

The loop talks to a backend with five operations (footprint, create, admit,
retire, step); `DeviceBackend` is the HIP library's.
"""
import collections
import dataclasses
import time

import numpy as np


class Arena:
    """First-fit allocator over [0, size) with 256-byte aligned blocks."""

    ALIGN = 256

    def __init__(self, size):
        self.size = int(size)
        self.free = [(0, self.size)]  # sorted (offset, length)
        self.used = {}

    def alloc(self, nbytes):
        n = (int(nbytes) + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        for k, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    del self.free[k]
                else:
                    self.free[k] = (off + n, ln - n)
                self.used[off] = n
                return off
        return None

    def release(self, off):
        n = self.used.pop(off)
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged

    @property
    def in_use(self):
        return sum(self.used.values())


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float
    problem: int
    m: int
    d: int
    N: int
    K: int
    seed: int
    gens: int
    op: str = "ga"  # reproduction operator: "ga", "de", "pso", "cso" or "rand"


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self):
        return self.finished - self.arrival


class DeviceBackend:
    """The HIP library: runs live in slices of one device arena."""

    def __init__(self, arena_bytes, max_runs, device="cuda:0", t_max=100, keep_state=False):
        import torch

        from . import rvea as R

        self.R = R
        self.torch = torch
        self.dev = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.dev)
        self.stream = torch.cuda.current_stream(self.dev)
        self.batch = R.Batch(max_runs, device=device, stream=self.stream)
        self.t_max = t_max
        self.keep_state = keep_state
        self.states = {}
        self._rid = {}

    def params(self, req):
        return self.R.default_params(req.op, t_max=max(self.t_max, req.gens))

    def footprint(self, req):
        return self.R.footprint(req.problem, req.m, req.d, req.N, req.K, self.params(req))

    def create(self, req, offset, nbytes):
        ws = self.arena.narrow(0, offset, nbytes)
        run = self.R.Run(req.problem, req.m, req.d, req.N, req.K, seed=req.seed,
                         params=self.params(req), device=self.dev, stream=self.stream,
                         workspace=ws)
        self._rid[id(run)] = req.rid
        return run

    def admit(self, run):
        self.batch.admit(run)

    def retire(self, run):
        self.batch.retire(run)
        if self.keep_state:
            self.states[self._rid[id(run)]] = run.get_state()
        self._rid.pop(id(run), None)
        run.close()

    # step(n) advances n ticks with one host synchronization at the end
    multi_tick = True

    def step(self, n=1):
        self.batch.step(n)
        self.batch.synchronize()


class Server:
    def __init__(self, backend, arena_bytes, max_runs):
        self.backend = backend
        self.arena = Arena(arena_bytes)
        self.max_runs = max_runs
        self.peak_runs = 0
        self.ticks = 0

    def serve(self, requests, clock=time.perf_counter, sleep=time.sleep):
        """Run every request to completion; returns Results in completion order."""
        queue = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        active = {}  # rid -> [request, run, offset, done, admitted]
        results = []
        t0 = clock()
        while queue or active:
            now = clock() - t0
            # admission: arrival order; the head waits until it fits
            while queue and queue[0].arrival <= now and len(active) < self.max_runs:
                req = queue[0]
                nb = self.backend.footprint(req)
                if nb + Arena.ALIGN > self.arena.size:
                    raise ValueError(f"request {req.rid} needs {nb} bytes, arena has "
                                     f"{self.arena.size}")
                off = self.arena.alloc(nb)
                if off is None:
                    break
                queue.popleft()
                run = self.backend.create(req, off, nb)
                self.backend.admit(run)
                active[req.rid] = [req, run, off, 0, now]
            if not active:
                if queue:
                    sleep(max(0.0, queue[0].arrival - (clock() - t0)))
                continue
            self.peak_runs = max(self.peak_runs, len(active))
            # with nothing left to admit, the ticks up to the next completion
            # go to the device at once (no host round trip between them)
            k = 1
            if not queue and getattr(self.backend, "multi_tick", False):
                k = min(ent[0].gens - ent[3] for ent in active.values())
            if k > 1:
                self.backend.step(k)
            else:
                self.backend.step()
            self.ticks += k
            now = clock() - t0
            for rid in list(active):
                ent = active[rid]
                ent[3] += k
                if ent[3] >= ent[0].gens:
                    req, run, off, _, adm = ent
                    self.backend.retire(run)
                    self.arena.release(off)
                    del active[rid]
                    results.append(Result(rid, req.arrival, adm, now))
        return results


def latency_summary(results, makespan=None):
    lat = np.array([r.latency for r in results])
    if makespan is None:
        makespan = max(r.finished for r in results) - min(r.arrival for r in results)
    return dict(runs=len(results), runs_per_s=len(results) / makespan,
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), makespan_s=makespan)
