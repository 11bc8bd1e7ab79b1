"""Serving driver: a stream of smoother requests on resident matrices.

The scheduling (admission by workspace footprint, continuous batching, one
batched launch per step) is native (``silu_server_*`` in libscaledilu.so);
this module builds the seeded request pool, feeds arrivals in real time, polls
completions, and reports latency percentiles beside throughput, against the
same requests run one at a time with ``ilu_smooth``.

Workload: 64 variable-density 7-point operators (no cut cells) with grid sides
drawn uniformly from {16, 24, 32, 48, 64, 96, 128} (seed 5), densities seeded
5 + j for matrix j, ILU(0) factors, row-scaled; 20 right-hand sides each,
b ~ U(-1, 1); 1,280 requests in shuffled order, each with 1-4 outer steps and
m_L = m_U = 3; Poisson arrivals at 2000 requests/s (seed 50).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B
from . import workloads as W

SIDES = (16, 24, 32, 48, 64, 96, 128)


@dataclass
class Request:
    mid: int
    b: torch.Tensor
    x: torch.Tensor
    outer: int
    m_L: int
    m_U: int
    arrival: float  # seconds after the start of the stream


def pool_spec(n_mat: int = 64, seed: int = 5, sides=SIDES):
    rng = np.random.default_rng(seed)
    return [int(s) for s in rng.choice(np.asarray(sides), size=n_mat)]


def build_pool(ctx: B.Context, sides, density_seed0: int = 5, fp32: bool = False):
    """Resident matrices: (A, factors) on the device for each side (fp32: the factors
    also carry FP32 values, for FP32-inner requests)."""
    mats = []
    for j, N in enumerate(sides):
        A = W.vardens7(N, seed_rho=density_seed0 + j, with_cuts=False)
        L, U = B.factor_iluk(A, 0)
        Ad, Ld, Ud = B.Csr.from_host(A), B.Csr.from_host(L), B.Csr.from_host(U)
        F = ctx.ilu_scale_factors(Ld, Ud, fp32=fp32)
        mats.append((Ad, F, A.n))
    return mats


def request_plan(n_mat: int, rhs_per_matrix: int = 20, rate: float = 2000.0, seed: int = 50, max_outer: int = 4):
    """The seeded request stream: (matrix id, rhs seed, outer steps, arrival time in s), in
    arrival order.  Shuffled (matrix, rhs) pairs; exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    order = [(mid, k) for mid in range(n_mat) for k in range(rhs_per_matrix)]
    perm = rng.permutation(len(order))
    gaps = rng.exponential(1.0 / rate, size=len(order))
    outers = rng.integers(1, max_outer + 1, size=len(order))
    t = np.cumsum(gaps)
    plan = []
    for i, p in enumerate(perm):
        mid, k = order[p]
        plan.append((mid, 1000 * mid + k, int(outers[i]), float(t[i])))
    return plan


def make_requests(mats, rhs_per_matrix: int = 20, rate: float = 2000.0, seed: int = 50, m: int = 3,
                  max_outer: int = 4):
    """All requests of the plan with their vectors resident on the device."""
    reqs = []
    for mid, bseed, outer, t in request_plan(len(mats), rhs_per_matrix, rate, seed, max_outer):
        n = mats[mid][2]
        b = torch.from_numpy(W.rhs(n, bseed)).cuda()
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        reqs.append(Request(mid, b, x, outer, m, m, t))
    return reqs


def run_batched(server: B.Server, mids, reqs, realtime: bool = True, lanes=None, steps_per_call: int = 1,
                mixed: bool = False):
    """Feed arrivals (in real time) to the server, step it, collect completions.
    lanes: optional list of (server, mids, max_rows) tried in order instead of
    the single server -- a request goes to the first lane whose max_rows covers
    its matrix, so each size class is batched on its own stream and small
    requests do not wait for the steps of large ones.  steps_per_call: scheduling
    steps per call into the library (silu_server_run), so the host loop does not
    pace the GPU.  mixed: every request in the FP32-inner form (the matrices' factors
    must carry FP32 values).  Returns (latencies in s, makespan in s, loop iterations)."""
    lanes = lanes or [(server, mids, None)]
    n = len(reqs)
    index = {}
    done_at = [0.0] * n
    pending = set()
    nxt = 0
    steps = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while nxt < n or pending:
        now = time.perf_counter() - t0
        while nxt < n and (not realtime or reqs[nxt].arrival <= now):
            r = reqs[nxt]
            li = next(k for k, (_, _, cap) in enumerate(lanes) if cap is None or r.b.numel() <= cap)
            sv, mv, _ = lanes[li]
            index[(li, sv.submit(mv[r.mid], r.b, r.x, r.outer, r.m_L, r.m_U, mixed=mixed))] = nxt
            pending.add(nxt)
            nxt += 1
        for li, (sv, _, _) in enumerate(lanes):
            if steps_per_call > 1:
                sv.run(steps_per_call)
            else:
                sv.step()
        steps += 1
        now = time.perf_counter() - t0
        for li, (sv, _, _) in enumerate(lanes):
            for t in sv.completed():
                i = index.pop((li, t))
                done_at[i] = now
                pending.discard(i)
        if not pending and nxt < n and realtime:
            wait = reqs[nxt].arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 1e-3))
    torch.cuda.synchronize()
    makespan = time.perf_counter() - t0
    lat = [done_at[i] - (reqs[i].arrival if realtime else 0.0) for i in range(n)]
    return np.asarray(lat), makespan, steps


def run_one_at_a_time(ctx: B.Context, mats, reqs, realtime: bool = True):
    """The same requests, each smoothed alone with ilu_smooth (FP64) in arrival order."""
    n = len(reqs)
    lat = np.zeros(n)
    ws = ctx.workspace(max(m[2] for m in mats))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        now = time.perf_counter() - t0
        if realtime and r.arrival > now:
            time.sleep(r.arrival - now)
        Ad, F, _ = mats[r.mid]
        ctx.ilu_smooth(Ad, F, r.b, r.x, r.outer, r.m_L, r.m_U, ws=ws)
        torch.cuda.synchronize()
        lat[i] = time.perf_counter() - t0 - (r.arrival if realtime else 0.0)
    makespan = time.perf_counter() - t0
    return lat, makespan


def percentiles(lat):
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(np.mean(lat) * 1e3)}
