"""Uneven batches: subtomograms of several box sizes (bandlimits) aligned in
one march.

Band indices are a prefix of the frequency order, so the coefficients of
every plan share the layout of any band L they contain.  The particles of
all box sizes are expanded (each with its own plan's basis) into the rows
of one coefficient array with a common stride, sorted by bandlimit, and
`bh_align_uneven` then runs one launch per band for every particle that
takes it: the bands are every `step` up to the largest bandlimit (plus each
box's own bandlimit), and a particle stops after its own.  Templates are
expanded per box size into rows of one template table.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence


@dataclass
class Group:
    """Particles of one box edge: vols [n, N, N, N] float32, template index
    per particle [n] (into that box's template list), starts [n, P, 3]."""
    N: int
    vols: object
    templates: object
    starts: object


class UnevenAligner:
    def __init__(self, plans: dict, templates: dict, step: int = 8):
        """plans: {N: Plan}; templates: {N: [T, C_N, 2] float32} with the same
        T for every N (template t rendered at each box size)."""
        import torch
        self.torch = torch
        self.plans = dict(plans)
        self.boxes = sorted(self.plans, key=lambda n: -self.plans[n].L_max)
        self.top = self.plans[self.boxes[0]]
        self.ld = self.top.C
        T = {int(t.shape[0]) for t in templates.values()}
        if len(T) != 1 or set(templates) != set(self.plans):
            raise ValueError("one template list of equal length per box edge")
        self.T = T.pop()
        dev = templates[self.boxes[0]].device
        self.table = torch.zeros((len(self.boxes) * self.T, self.ld, 2), dtype=torch.float32,
                                 device=dev)
        for k, n in enumerate(self.boxes):
            C = self.plans[n].C
            self.table[k * self.T:(k + 1) * self.T, :C] = templates[n]
        Ls = sorted({self.plans[n].L_max for n in self.boxes})
        self.bands = sorted(set(range(step, Ls[-1] + 1, step)) | set(Ls))

    def align(self, groups: Sequence[Group], steps: int, mode: str = "fp32",
              batch_invariant: bool = False, **opts):
        """Best rotation and score per particle, returned per group in the
        order given: [(euler [n, 3], score [n]), ...]."""
        a, Lp, tmpl, bands, starts, rows = self.pack(groups, mode, batch_invariant)
        eu, sc = self.top.align_uneven(a, Lp, self.table, tmpl, bands, starts, steps,
                                       batch_invariant=batch_invariant, **opts)
        return [(eu[rows[i][0]:rows[i][1]], sc[rows[i][0]:rows[i][1]])
                for i in range(len(groups))]

    def pack(self, groups: Sequence[Group], mode: str = "fp32", batch_invariant: bool = False):
        """The inputs of one uneven march: (a [n, ld, 2], Lp, template index
        [n] int32, bands, starts [n, P, 3], {group: (first row, end row)}),
        rows sorted by bandlimit."""
        torch = self.torch
        order = sorted(range(len(groups)), key=lambda i: -self.plans[groups[i].N].L_max)
        n_tot = sum(int(groups[i].vols.shape[0]) for i in order)
        dev = self.table.device
        a = torch.zeros((n_tot, self.ld, 2), dtype=torch.float32, device=dev)
        Lp, tmpl, starts, rows = [], [], [], {}
        r0 = 0
        for i in order:
            g = groups[i]
            n = int(g.vols.shape[0])
            plan = self.plans[g.N]
            plan.expand_into(g.vols, a[r0:r0 + n], mode=mode, batch_invariant=batch_invariant)
            k = self.boxes.index(g.N)
            tmpl.append(torch.as_tensor(g.templates, dtype=torch.int32, device=dev) + k * self.T)
            starts.append(g.starts)
            Lp += [plan.L_max] * n
            rows[i] = (r0, r0 + n)
            r0 += n
        first = [b for b in self.bands if b <= min(Lp)]
        bands = [b for b in self.bands if b >= (first[0] if first else self.bands[0])]
        return (a, Lp, torch.cat(tmpl).contiguous(), bands, torch.cat(starts).contiguous(), rows)
