"""HIP-graph capture of marching calls (one template table or uneven batches).

A marching call issues a fixed sequence of launches per band (class weights
and step scale, ascent kernel) and a selection; for repeated calls on
buffers of a fixed shape the whole sequence can be captured once and
replayed, which removes the per-launch host cost (it matters for small
batches, where each launch is short).  Capture happens on a side stream
after one eager warm-up call, so that every scratch buffer and band table
already exists: nothing is allocated or uploaded while capturing, and no
memset nodes are recorded (the library clears nothing with memset).
"""

from __future__ import annotations

from typing import Sequence


class GraphedAlign:
    """bh_align_t on fixed buffers, captured once and replayed.

    a [B, C, 2], templates [T, C, 2], tmpl_idx [B] or None, starts [B, P, 3]
    keep their addresses; refill them in place between replays.  Results land
    in self.euler [B, 3] and self.score [B].
    """

    def __init__(self, plan, a, templates, tmpl_idx, bands: Sequence[int], starts, steps: int,
                 **opts):
        import torch
        self.torch = torch
        B = a.shape[0]
        self.euler = torch.empty((B, 3), dtype=torch.float64, device=a.device)
        self.score = torch.empty((B,), dtype=torch.float64, device=a.device)
        args = (a, templates, tmpl_idx, list(bands), starts, steps)
        out = (self.euler, self.score, None, None)
        plan.align_t(*args, out=out, **opts)              # warm-up: scratch and tables
        torch.cuda.synchronize(a.device)
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=a.device)
        side.wait_stream(torch.cuda.current_stream(a.device))
        with torch.cuda.stream(side):
            with torch.cuda.graph(self.graph, stream=side):
                plan.align_t(*args, out=out, **opts)
        torch.cuda.current_stream(a.device).wait_stream(side)

    def replay(self):
        self.graph.replay()
        return self.euler, self.score


class GraphedAlignUneven:
    """bh_align_uneven on fixed buffers (the rows of all box sizes in one
    coefficient array, bandlimits non-increasing), captured once and
    replayed; as GraphedAlign, refill a and starts in place between replays.
    Results land in self.euler [B, 3] and self.score [B]."""

    def __init__(self, plan, a, Lp, templates, tmpl_idx, bands: Sequence[int], starts, steps: int,
                 **opts):
        import torch
        self.torch = torch
        B = a.shape[0]
        self.euler = torch.empty((B, 3), dtype=torch.float64, device=a.device)
        self.score = torch.empty((B,), dtype=torch.float64, device=a.device)
        self.Lp = list(int(x) for x in Lp)
        args = (a, self.Lp, templates, tmpl_idx, list(bands), starts, steps)
        out = (self.euler, self.score, None, None)
        plan.align_uneven(*args, out=out, **opts)         # warm-up: scratch and tables
        torch.cuda.synchronize(a.device)
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=a.device)
        side.wait_stream(torch.cuda.current_stream(a.device))
        with torch.cuda.stream(side):
            with torch.cuda.graph(self.graph, stream=side):
                plan.align_uneven(*args, out=out, **opts)
        torch.cuda.current_stream(a.device).wait_stream(side)

    def replay(self):
        self.graph.replay()
        return self.euler, self.score
