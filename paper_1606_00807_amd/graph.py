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

This module only orders and captures library calls: the arithmetic is the
library's.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

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
        self.streams = [torch.cuda.Stream() for _ in range(self.branches)]
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
