"""Serving loop: assembly requests on resident geometries, with continuous
batching and admission by an HBM budget.

A request asks for the matrices of one resident patch (geometry) for a new
diffusion coefficient a(x).  Each geometry is a bound plan set up once for
a = 1: its univariate rules (weights, operator tables), det J and J^{-1} at
the quadrature points, its physical points and its CSR pattern stay in
device memory.  A request only evaluates its coefficient at the resident
points and calls ``wq_assemble_request`` with a request context (coefficient
field and first-contraction buffer) and outputs of its own, so requests on
the same geometry overlap freely.

Continuous batching: requests that arrive while others are on the device
are admitted as soon as an in-flight slot and enough of the memory budget
are free, and their work is issued at once on one of a few HIP streams, so
it overlaps with the work already in flight; completions are detected by
events and free their slot and memory.  Every step of the method runs in
the HIP library; this module only schedules calls.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import WQ_FP32, WQ_MASS, WQ_STIFF, Plan


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival: float     # seconds from the start of the run
    geom: int          # index of a resident geometry
    coef_seed: int     # seed of the request's coefficient field


@dataclasses.dataclass
class Record:
    rid: int
    geom: int
    arrival: float
    admitted: float
    done: float
    nnz: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Geometry:
    """One resident patch: a plan set up for a = 1, its physical quadrature
    points (to evaluate request coefficients) and its CSR pattern."""

    def __init__(self, knots, p: int, ctrl_np: np.ndarray, precision: int = WQ_FP32,
                 which: int = WQ_STIFF):
        import torch
        self.plan = Plan(knots, p, precision)
        self.plan.bind()
        self.plan.setup(torch.from_numpy(np.ascontiguousarray(ctrl_np)).cuda())
        self.xq = self.plan.qp_physical().reshape(-1, self.plan.d)
        self.row_ptr, self.col_idx = self.plan.pattern()
        self.plan.sync()
        self.which = which
        self.n_mat = (1 if which & WQ_MASS else 0) + (1 if which & WQ_STIFF else 0)
        self.ctx_bytes = self.plan.request_bytes() + 256
        elem = 8 if self.plan.value_dtype == torch.float64 else 4
        self.out_bytes = self.plan.nnz * elem * self.n_mat

    @property
    def bytes_per_request(self) -> int:
        return self.ctx_bytes + self.out_bytes


def poisson_requests(n: int, rate: float, n_geoms: int, seed: int) -> List[Request]:
    """n requests with exponential inter-arrival times of mean 1/rate
    (rate <= 0: all arrive at t = 0), geometry uniform over n_geoms, a fresh
    coefficient seed each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n)) if rate > 0 else np.zeros(n)
    g = rng.integers(0, n_geoms, size=n)
    return [Request(k, float(t[k]), int(g[k]), int(seed * 100003 + k)) for k in range(n)]


class Server:
    """Continuous-batching request loop over resident geometries.

    coef_fn(request, xq) -> device float64 tensor of a at the points xq
    (n_qp_total x d, on the device), evaluated on the request's stream."""

    def __init__(self, geoms: Sequence[Geometry], coef_fn: Callable, n_streams: int = 4,
                 max_inflight: int = 16, hbm_budget: int = 16 << 30):
        import torch
        self.geoms = list(geoms)
        self.coef_fn = coef_fn
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.max_inflight = max_inflight
        self.hbm_budget = hbm_budget
        self.peak_bytes = 0
        self.peak_inflight = 0

    def _launch(self, req: Request, stream):
        import torch
        g = self.geoms[req.geom]
        with torch.cuda.stream(stream):
            ctx = torch.empty(g.ctx_bytes, dtype=torch.uint8, device="cuda")
            coef = self.coef_fn(req, g.xq)
            mass, stiff = g.plan.assemble_request(ctx, coef, g.which, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev, (ctx, coef, mass, stiff)

    def run(self, requests: Sequence[Request], keep: Optional[set] = None) -> Dict:
        """Serve the requests (arrival times relative to the start of the
        call).  Returns the records and, for request ids in ``keep``, the
        output tensors (mass, stiff)."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        inflight = []
        records: List[Record] = []
        outputs = {}
        used = 0
        k = 0
        t0 = time.perf_counter()
        while pending or inflight:
            now = time.perf_counter() - t0
            still = []
            for req, ev, bufs, admitted, nbytes in inflight:
                if ev.query():
                    g = self.geoms[req.geom]
                    records.append(Record(req.rid, req.geom, req.arrival, admitted, now, g.plan.nnz * g.n_mat))
                    used -= nbytes
                    if keep is not None and req.rid in keep:
                        outputs[req.rid] = (bufs[2], bufs[3])
                else:
                    still.append((req, ev, bufs, admitted, nbytes))
            inflight = still
            while pending and pending[0].arrival <= now and len(inflight) < self.max_inflight:
                req = pending[0]
                need = self.geoms[req.geom].bytes_per_request
                if used + need > self.hbm_budget and inflight:
                    break   # wait until enough memory is free
                pending.popleft()
                ev, bufs = self._launch(req, self.streams[k % len(self.streams)])
                k += 1
                used += need
                inflight.append((req, ev, bufs, time.perf_counter() - t0, need))
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_inflight = max(self.peak_inflight, len(inflight))
        wall = time.perf_counter() - t0
        return {"records": records, "outputs": outputs, "wall_s": wall}

    def serve_alone(self, req: Request):
        """One request with nothing else in flight (the reference of the
        alone-vs-mix test)."""
        ev, bufs = self._launch(req, self.streams[0])
        ev.synchronize()
        return bufs[2], bufs[3]


def summarize(result: Dict) -> Dict:
    recs = result["records"]
    lat = np.array([r.latency for r in recs]) * 1e3
    nnz = sum(r.nnz for r in recs)
    wall = result["wall_s"]
    return {"requests": len(recs), "wall_s": round(wall, 4),
            "requests_per_s": round(len(recs) / wall, 2),
            "gnnz_per_s": round(nnz / wall / 1e9, 3),
            "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
            "latency_ms_p99": round(float(np.percentile(lat, 99)), 4)}
