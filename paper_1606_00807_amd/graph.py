"""Many independent EnKF-MC problems (each its own Plan) assimilated by one
HIP graph launch.

Every plan runs in asynchronous mode, so its enkfmc_fit and enkfmc_analyze
calls only enqueue kernels and can be captured.  The instances are spread
over a few branches of the graph (longest-first onto the least-loaded
branch, by the fit's leading cost n_fit * min(p, N)^2 with p ~ the plan's
largest predecessor count), each branch running its instances one after the
other; the branches run concurrently.  A device timestamp is written before
an instance's first kernel and after its last, so each replay gives every
instance's latency from the device clock.

The branches run on streams of their own, created for the graph: streams
taken from torch's pool may share a hardware queue with each other once
the process has used many streams, and two branches on one queue run one
after the other.

This module only orders and captures library calls: the arithmetic is the
library's.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from ._lib import hip_stream_create, hip_stream_destroy
from .api import Plan, timestamp, wall_clock_hz


class InstanceGraph:
    """items: sequence of dicts with keys plan (Plan), Xb (CUDA tensor), Y,
    r_diag (CUDA float64 tensors), ridge (float), and optionally mode
    ("batched" by default)."""

    def __init__(self, items: Sequence[Dict], branches: int = 4):
        import torch
        self.items = list(items)
        self.branches = max(1, min(int(branches), len(self.items)))
        n = len(self.items)
        for it in self.items:
            it["plan"].ensure_workspace()
            it["plan"].set_async(True)
        self.ts = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
        self.hz = wall_clock_hz()
        # longest first onto the least-loaded branch
        cost = [self._cost(it["plan"]) for it in self.items]
        load = [0.0] * self.branches
        self.assign: List[List[int]] = [[] for _ in range(self.branches)]
        for k in sorted(range(n), key=lambda k: -cost[k]):
            b = int(np.argmin(load))
            self.assign[b].append(k)
            load[b] += cost[k]
        self._raw_streams = [hip_stream_create() for _ in range(self.branches)]
        self.streams = [torch.cuda.ExternalStream(h) for h in self._raw_streams]
        self.Xa: List = [None] * n
        self.graph = None

    @staticmethod
    def _cost(plan: Plan) -> float:
        m = min(plan.info["max_p"], plan.N)
        return float(plan.info["n_fit"]) * (m * m + plan.N)

    def _enqueue(self) -> None:
        import torch
        main = torch.cuda.current_stream()
        for b, s in enumerate(self.streams):
            s.wait_stream(main)
            with torch.cuda.stream(s):
                for k in self.assign[b]:
                    it = self.items[k]
                    plan = it["plan"]
                    timestamp(self.ts[k, 0])
                    plan.fit(it["Xb"], it["ridge"], mode=it.get("mode", "batched"))
                    self.Xa[k] = plan.analyze(it["Xb"], it["Y"], it["r_diag"])
                    timestamp(self.ts[k, 1])
        for s in self.streams:
            main.wait_stream(s)

    def run_eager(self) -> List:
        """The same calls without a graph (asynchronous plans on the branch
        streams); returns the analyses."""
        import torch
        self._enqueue()
        torch.cuda.synchronize()
        self.check()
        return [x.clone() for x in self.Xa]

    def capture(self) -> None:
        import torch
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._enqueue()
        torch.cuda.synchronize()

    def replay(self) -> None:
        self.graph.replay()

    def check(self) -> None:
        """Raise the first device-side failure of any instance (synchronises)."""
        for it in self.items:
            it["plan"].check_status()

    def latencies_ms(self) -> np.ndarray:
        """Per-instance latency of the last run, from the device clock."""
        t = self.ts.cpu().numpy()
        return (t[:, 1] - t[:, 0]) / self.hz * 1e3

    def close(self) -> None:
        for it in self.items:
            it["plan"].set_async(False)
        self.graph = None
        self.streams = []
        for h in self._raw_streams:
            hip_stream_destroy(h)
        self._raw_streams = []


def _tune_key(items: Sequence[Dict]) -> str:
    """Device architecture and a digest of the instance set (each plan's n,
    N, largest predecessor count, regressions, observations and fit mode)."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName
    sig = sorted((int(it["plan"].info["n"]), int(it["plan"].N), int(it["plan"].info["max_p"]),
                  int(it["plan"].info["n_fit"]), int(it["plan"].info["m"]), str(it.get("mode", "batched")))
                 for it in items)
    return arch + ":" + hashlib.sha1(repr(sig).encode()).hexdigest()[:16]


def tune_branches(items: Sequence[Dict], candidates: Sequence[int] = (1, 2, 4, 8, 16), reps: int = 3,
                  cache: Optional[str] = None) -> Tuple[int, Dict[int, float]]:
    """Branch count of an InstanceGraph for these instances: each candidate's
    eager run (the same enqueue order on the branch streams, no graph) timed
    by events, median of reps after one warm-up; the fastest wins.  With a
    cache file (JSON), a result for the same device architecture and
    instance set is reused and new results are stored; an unreadable or
    unwritable cache is ignored.  Returns (branches, ms per candidate)."""
    import torch
    key = _tune_key(items)
    table: Dict = {}
    if cache:
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
        hit = table.get(key)
        if isinstance(hit, dict) and "branches" in hit:
            return int(hit["branches"]), {int(k): float(v) for k, v in hit.get("ms", {}).items()}
    times: Dict[int, float] = {}
    for b in candidates:
        if b > len(items):
            continue
        g = InstanceGraph(items, branches=b)
        g.run_eager()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            ev0.record()
            g._enqueue()
            ev1.record()
            torch.cuda.synchronize()
            ms.append(ev0.elapsed_time(ev1))
        g.check()
        g.close()
        times[b] = float(np.median(ms))
    best = min(times, key=times.get)
    if cache:
        table[key] = {"branches": best, "ms": {str(k): v for k, v in times.items()}}
        try:
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        except OSError:
            pass
    return best, times
