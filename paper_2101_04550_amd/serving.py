"""Continuous-batching request server for lattice solves on one GPU.

Requests (a lattice, its initial fields and a step count) arrive over time.
The server admits arrived requests in arrival order while their device
footprint (``elbm_query_bytes``) fits the memory budget and a slot is free,
keeps the admitted lattices resident, and advances all of them together in
rounds: each round is one ``elbm_batch_run`` of up to ``quantum`` steps per
lattice, i.e. per step one fused launch per kernel class over the tiles of
every resident lattice, replayed from a cached HIP graph. Requests that
arrive while others are on the GPU join at the next round; finished lattices
are read back and released at once, freeing memory and slots.

Every lattice advances bitwise as it would alone (the batched launch runs the
same kernel on the same tiles), so a served result equals a solo run.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import elbm as E


@dataclass
class Request:
    """One solve: lattice parameters, initial fields and a step count."""
    rid: int
    kind: str
    n: tuple
    lam: tuple
    T: float
    omega: float
    steps: int
    storage: str
    arrival: float
    u_adv: tuple = None
    rho: np.ndarray = None
    u: np.ndarray = None

    def params(self):
        return E.make_params(self.n, lam=self.lam, T=self.T, omega=self.omega, u_adv=self.u_adv,
                             storage=self.storage)

    @property
    def cells(self):
        return int(math.prod(self.n))


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    cells: int
    ke: float
    enstrophy: float
    min_rho: float
    checksum: str
    rho: np.ndarray = None  # final fields, kept when the server is asked to (keep_fields)
    u: np.ndarray = None

    @property
    def latency(self):
        return self.finished - self.arrival


def state_checksum(lat) -> str:
    """sha256 of the lattice's raw stored state (bitwise identity of a result)."""
    return hashlib.sha256(lat.save().tobytes()).hexdigest()


@dataclass
class _Active:
    req: Request
    lat: object
    remaining: int
    admitted: float
    nbytes: int


class Server:
    """Admission by device footprint, resident lattices, graph-replayed fused rounds."""

    def __init__(self, pool_bytes: int, max_slots: int = 64, quantum: int = 100, use_graph: bool = True,
                 checksums: bool = False, keep_fields: bool = False):
        import torch

        self.torch = torch
        self.pool_bytes = int(pool_bytes)
        self.max_slots = int(max_slots)
        self.quantum = int(quantum)
        self.use_graph = bool(use_graph)
        self.checksums = bool(checksums)
        self.keep_fields = bool(keep_fields)
        self.batch = E.Batch(self.max_slots)
        # one stream per resident lattice: its upload at admission is ordered
        # after nothing else, so it runs while a round is on the GPU (the
        # batch orders each round after the lattices' streams itself)
        self.streams = [torch.cuda.Stream() for _ in range(self.max_slots)]
        self.used = 0
        self.rounds = 0
        self.peak_used = 0
        self.peak_slots = 0

    def close(self):
        self.batch.close()

    def _admit(self, req: Request, now: float):
        p = req.params()
        nbytes = E.query_bytes(p)
        stream = self.streams.pop()
        lat = E.Lattice(p, stream=stream)
        lat.init(req.rho, req.u)
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        return _Active(req, lat, req.steps, now, nbytes)

    def _release(self, a):
        a.lat.close()
        self.streams.append(a.lat.stream)
        self.used -= a.nbytes

    def fits(self, req: Request, nactive: int) -> bool:
        return nactive < self.max_slots and self.used + E.query_bytes(req.params()) <= self.pool_bytes

    def run(self, requests, clock=time.perf_counter):
        """Serves `requests` (arrival times in seconds from the start); returns results by rid.

        Each round launches one batched run of up to `quantum` steps for every
        resident lattice; while the GPU works, newly arrived requests are
        admitted (their fields uploaded) and join the next round."""
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        for r in pending:
            if E.query_bytes(r.params()) > self.pool_bytes:
                raise ValueError(f"request {r.rid} needs more device memory than the whole budget")
        waiting = deque()
        active = []
        results = {}
        t0 = clock()

        def admit_arrived(nresident):
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            joined = []
            while waiting and self.fits(waiting[0], nresident + len(joined)):
                joined.append(self._admit(waiting.popleft(), clock() - t0))
            return joined

        while pending or waiting or active:
            active += admit_arrived(len(active))
            self.peak_slots = max(self.peak_slots, len(active))
            if not active:
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - (clock() - t0), 0.01)))
                continue
            steps = [min(self.quantum, a.remaining) for a in active]
            self.batch.run([a.lat for a in active], steps, use_graph=self.use_graph)
            self.rounds += 1
            # overlap: admit arrivals while the round runs (they join the next round)
            joined = admit_arrived(len(active))
            self.torch.cuda.synchronize()
            done_at = clock() - t0
            still = []
            for a, s in zip(active, steps):
                a.remaining -= s
                if a.remaining > 0:
                    still.append(a)
                    continue
                d = a.lat.diag(check=False)
                cs = state_checksum(a.lat) if self.checksums else ""
                rho, u = a.lat.fields() if self.keep_fields else (None, None)
                results[a.req.rid] = Result(a.req.rid, a.req.arrival, a.admitted, done_at, a.req.steps,
                                            a.req.cells, d["ke"], d["enstrophy"], d["min_rho"], cs, rho, u)
                self._release(a)
            active = still + joined
            self.peak_slots = max(self.peak_slots, len(active))
        self.makespan = clock() - t0
        return results


def summarize(results, makespan):
    lat = np.array(sorted(r.latency for r in results.values()))
    updates = sum(r.cells * r.steps for r in results.values())
    return {
        "requests": len(results),
        "makespan_s": makespan,
        "solves_per_s": len(results) / makespan,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "sustained_glups": updates / makespan / 1e9,
        "cell_updates": updates,
    }


# ---------------------------------------------------------------------------
# The mixed request stream (seeded): shear waves and double shear layers on
# D2Q9, decaying turbulence boxes on D3Q27.
# ---------------------------------------------------------------------------

SIZES_2D = (64, 128, 256, 512, 1024)
SIZES_3D = (64, 96, 128, 160, 192)


def _omega(nu, T):
    return 1.0 / (nu / T + 0.5)


def make_stream(count=600, rate=50.0, share_3d=0.1, seed_offset=5, steps_range=(200, 5000)):
    """Seeded Poisson stream: kind, size, T in {1/3, 1/2}, stretch in {1, 0.5},
    log-uniform steps, FP32 / FP16 storage 50/50. Fields are attached later."""
    import inputs as I

    g = I.rng(seed_offset)
    t = 0.0
    reqs = []
    for rid in range(count):
        t += g.exponential(1.0 / rate)
        T = (1.0 / 3.0, 0.5)[int(g.integers(0, 2))]
        stretched = bool(g.integers(0, 2))
        steps = int(round(math.exp(g.uniform(math.log(steps_range[0]), math.log(steps_range[1])))))
        storage = ("f32", "f16")[int(g.integers(0, 2))]
        if g.random() < share_3d:
            N = int(SIZES_3D[int(g.integers(0, len(SIZES_3D)))])
            n = (N // 2, N, N) if stretched else (N, N, N)
            lam = (2.0, 1.0, 1.0) if stretched else (1.0, 1.0, 1.0)
            lam_T = N / (4.0 * math.pi)  # Taylor microscale of the k0 = 4 spectrum
            nu = 0.05 * lam_T / 72.0
            reqs.append(Request(rid, "hit", n, lam, T, _omega(nu, T), steps, storage, t))
        else:
            N = int(SIZES_2D[int(g.integers(0, len(SIZES_2D)))])
            n = (N // 2, N) if stretched else (N, N)
            lam = (2.0, 1.0) if stretched else (1.0, 1.0)
            if g.random() < 0.5:
                reqs.append(Request(rid, "shear", n, lam, T, 1.8, steps, storage, t, u_adv=(0.1, 0.0)))
            else:
                nu = 0.1 * 1024 / 30000.0  # Re = 30000 N / 1024 at U = 0.1, L = N
                reqs.append(Request(rid, "dsl", n, lam, T, _omega(nu, T), steps, storage, t))
    return reqs


def attach_fields(reqs):
    """Initial fields of every request (seeded, cached by kind / shape / stretch)."""
    import inputs as I

    cache = {}
    for r in reqs:
        key = (r.kind, r.n, r.lam)
        if key not in cache:
            if r.kind == "shear":
                f = I.shear_wave_axis(r.n, U0=0.0, A=0.01, lam=r.lam)
            elif r.kind == "dsl":
                f = I.double_shear_layer(r.n, lam=r.lam)
            else:
                N = r.n[1]
                f = I.hit_field(N, k0=4.0, urms=0.05)
                if r.n[0] != N:  # stretched box: every second x node of the cubic field
                    f = I.Field(f.rho[:, :, ::2].copy(), f.u[:, :, :, ::2].copy(), r.n, r.lam)
            cache[key] = (np.ascontiguousarray(f.rho), np.ascontiguousarray(f.u))
        r.rho, r.u = cache[key]
    return reqs


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--requests", type=int, default=600)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--share-3d", type=float, default=0.1)
    ap.add_argument("--pool-gb", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--quantum", type=int, default=100)
    ap.add_argument("--no-graph", action="store_true")
    args = ap.parse_args(argv)
    reqs = attach_fields(make_stream(args.requests, args.rate, args.share_3d))
    offered = sum(r.cells * r.steps for r in reqs)
    srv = Server(int(args.pool_gb * 2 ** 30), args.slots, args.quantum, not args.no_graph)
    res = srv.run(reqs)
    out = summarize(res, srv.makespan)
    out.update({"offered_cell_updates": offered, "arrival_window_s": reqs[-1].arrival, "rounds": srv.rounds,
                "peak_slots": srv.peak_slots, "peak_pool_gb": srv.peak_used / 2 ** 30,
                "share_3d": args.share_3d, "rate": args.rate, "quantum": args.quantum})
    srv.close()
    print(json.dumps(out))


if __name__ == "__main__":
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    main()
