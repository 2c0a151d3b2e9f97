"""Continuous-batching alignment server on one GPU.

Requests (subtomograms of one box edge, matched against one of several
resident templates) queue on arrival and are served in ticks.  One tick:

1. Admission.  In arrival order, queued requests join a new cohort of their
   box edge while the device-memory budget allows (and the cohort stays
   under its size cap); admission stops at the first request that does not
   fit, so no request is overtaken.  The new cohort's volumes are expanded
   once (split-BF16 MFMA expansion, Sec. II-A: the BF16 coefficients for the
   coarse bands and the refined, near-FP32 ones for the final band) and its
   starting rotations are loaded; from then on the cohort's coefficients
   and the restarts' angles (the optimiser state) stay on the device.
   Requests that name rows of one resident volume stack (Rows) are expanded
   from it in place; others are first copied into one cohort array.
2. Marching.  Every live cohort advances by one band of the frequency march
   (Sec. II-C): the gradient-ascent steps of that band for all of its
   restarts, against each particle's own template.  Cohorts admitted at
   the same tick always share their band, so each (box, band) batch is one
   contiguous cohort and requests never need to be gathered.
3. Completion.  A cohort past its last band hands each request its best
   rotation and score and releases its share of the budget.

New requests therefore join between marching steps while earlier ones are
still on the GPU.  Each box edge has its own plan and HIP stream (default
priority), so the work of different box sizes overlaps on the device.  The
expansion and the march run in their batch-invariant forms, so a
particle's result is bit-for-bit the same alone and in any mix.

The host logic (admission, cohort bookkeeping) is in Scheduler, which needs
no GPU; Engine drives the library through the Python binding.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np


# ------------------------------------------------------------- host logic --

@dataclass
class BoxSpec:
    """How one box edge is served: bandlimit, marching bands and the device
    bytes one particle holds while in flight."""
    N: int
    L_max: int
    bands: tuple
    bytes_per_particle: int


@dataclass
class Rows:
    """A request's particles as rows of a resident volume stack: particle i
    is stack[index[i]].  stack: [n_vols, N, N, N] float32 device tensor;
    index: [n] int64 tensor (device, or host: then range-checked at
    submission and copied to the device asynchronously at admission).  The
    expansion reads the rows in place, at admission on the engine's stream:
    they must not change until the request's cohort has been admitted and
    expanded (its results returned is a safe point).  A device index outside
    the stack gives NaN results for those particles and BhError (BH_EINVAL)
    from the engine's next library call on that box edge."""
    stack: object
    index: object


@dataclass
class Request:
    """One alignment request.

    volumes: [n, N, N, N] float32 device tensor, Rows, or a callable
             returning either (called once, at admission).
    starts:  [n, P, 3] float64 device tensor of starting Euler triples, or a
             callable returning it.
    arrival: time.perf_counter() at submission (set by submit if None).
    """
    box: int
    template: int
    n: int
    volumes: object
    starts: object
    rid: int = -1
    arrival: float | None = None
    admitted: float | None = None
    done: float | None = None
    euler: np.ndarray | None = None     # [n, 3] best rotation (ZYZ Euler)
    score: np.ndarray | None = None     # [n] its score


@dataclass
class Cohort:
    """Requests admitted together for one box edge; `bands` is its march
    schedule, the box's at admission."""
    box: int
    requests: list
    n: int
    nbytes: int
    tick: int
    cursor: int = 0                     # index of the next band to run
    bands: tuple = ()
    dev: dict = field(default_factory=dict)


class Scheduler:
    """Admission and cohort bookkeeping (no device work)."""

    def __init__(self, specs: dict, budget_bytes: int, max_cohort: int = 2048):
        self.specs = dict(specs)
        self.budget = int(budget_bytes)
        self.max_cohort = int(max_cohort)
        self.queue: deque = deque()
        self.live: list = []
        self.used = 0
        self.ticks = 0

    def submit(self, req: Request) -> None:
        spec = self.specs.get(req.box)
        if spec is None:
            raise ValueError(f"no plan serves box edge {req.box}")
        if req.n < 1:
            raise ValueError("a request needs at least one particle")
        if req.n * spec.bytes_per_particle > self.budget:
            raise ValueError(f"request of {req.n} particles at {req.box}^3 exceeds the budget")
        self.queue.append(req)

    def admit(self) -> list:
        """Form this tick's new cohorts (one per box edge at most)."""
        new: dict = {}
        while self.queue:
            r = self.queue[0]
            need = r.n * self.specs[r.box].bytes_per_particle
            if self.used + need > self.budget:
                break
            c = new.get(r.box)
            if c is not None and c.n + r.n > self.max_cohort:
                break
            self.queue.popleft()
            if c is None:
                c = new[r.box] = Cohort(box=r.box, requests=[], n=0, nbytes=0, tick=self.ticks,
                                        bands=self.specs[r.box].bands)
            c.requests.append(r)
            c.n += r.n
            c.nbytes += need
            self.used += need
        cohorts = list(new.values())
        self.live.extend(cohorts)
        return cohorts

    def plan(self) -> list:
        """(cohort, band, is_last) for every live cohort, in admission order."""
        out = []
        for c in self.live:
            out.append((c, c.bands[c.cursor], c.cursor == len(c.bands) - 1))
        return out

    def advance(self) -> list:
        """Move every live cohort past its band; return the finished ones."""
        done, keep = [], []
        for c in self.live:
            c.cursor += 1
            if c.cursor == len(c.bands):
                done.append(c)
                self.used -= c.nbytes
            else:
                keep.append(c)
        self.live = keep
        self.ticks += 1
        return done

    def busy(self) -> bool:
        return bool(self.queue or self.live)

    def queued_particles(self) -> int:
        return sum(r.n for r in self.queue)


# ----------------------------------------------------------------- engine --

def _band_entries(L: int) -> int:
    # (m >= |n|) class entries of band L: sum over m of (2m+1) classes of
    # L-m+1 degrees each, plus the table padding.
    return sum((2 * m + 1) * (L - m + 1) for m in range(L + 1)) + 4


class Engine:
    """The serving loop on one GPU.

    boxes:     {N: (L_max, bands)}
    templates: {N: [T, C(L_max), 2] float32 device tensor} resident
               template coefficients per box edge
    """

    def __init__(self, boxes: dict, templates: dict, restarts: int, steps: int,
                 budget_bytes: int = 24 << 30, max_cohort: int = 2048, device: int = 0,
                 step_init: float = 1.0, step_grow: float = 1.25, step_shrink: float = 0.5,
                 plans: dict | None = None, method: str = "march", keep: int = 8,
                 min_sep: float = 0.17453292519943295, newton_steps: int = 6,
                 band_thresholds: Sequence[float] | None = None):
        """method "march": gradient steps on every band; "paper": after the
        first band only `keep` candidates (local maxima at least `min_sep`
        radians apart) continue, with `newton_steps` Newton steps per band.

        band_thresholds: choose each box edge's march schedule by the
        energy ratio (bh_select_bands, Fig. 1 caption and Sec. III) instead
        of the given bands: each resident template's cross-power with
        itself up to the box's largest band, the batch choice over the
        templates for these thresholds, then that band.  It is chosen once,
        here, from the templates only, so a request's result still does not
        depend on the requests it is served with (a choice per cohort from
        the particles would)."""
        import torch
        from .api import Plan
        if method not in ("march", "paper"):
            raise ValueError("method is 'march' or 'paper'")
        self.method, self.keep, self.min_sep = method, int(keep), float(min_sep)
        self.band_thresholds = (None if band_thresholds is None
                                else tuple(float(t) for t in band_thresholds))
        self.newton_steps = int(newton_steps)
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.P, self.steps = int(restarts), int(steps)
        self.step_args = (float(step_init), float(step_grow), float(step_shrink))
        self.plans = {}
        self.streams = {}
        specs = {}
        for N, (L, bands) in boxes.items():
            plan = (plans or {}).get(N) or Plan(N, L, device=device)
            if plan.L_max != L:
                raise ValueError(f"plan for {N}^3 has L_max {plan.L_max}, not {L}")
            if max(bands) > L:
                raise ValueError(f"bands of {N}^3 exceed its bandlimit {L}")
            # the engine overlaps work across its own per-box streams; each
            # band march stays on its box stream (no split over a plan stream)
            plan.set_march_streams(1)
            self.plans[N] = plan
            self.streams[N] = torch.cuda.Stream(device=self.dev)
            specs[N] = BoxSpec(N, L, tuple(int(b) for b in bands),
                               self.particle_bytes(plan, max(bands)))
        self.templates = {}
        for N, t in templates.items():
            if N not in self.plans:
                raise ValueError(f"templates given for unserved box edge {N}")
            if t.dtype != torch.float32 or t.dim() != 3 or t.shape[1:] != (self.plans[N].C, 2):
                raise ValueError(f"templates of {N}^3 must be [T, {self.plans[N].C}, 2] float32")
            self.templates[N] = t.contiguous()
        # the templates may still be in flight on the caller's stream
        cur = torch.cuda.current_stream(self.dev)
        for N, s in self.streams.items():
            s.wait_stream(cur)
            if N in self.templates:
                self.templates[N].record_stream(s)
        if self.band_thresholds is not None:
            for N, spec in specs.items():
                if N not in self.templates:
                    continue
                t = self.templates[N]
                ti = torch.arange(t.shape[0], dtype=torch.int32, device=self.dev)
                L_top = max(spec.bands)
                _b, common, _r = self.plans[N].select_bands(t, t, ti, L_top, self.band_thresholds)
                spec.bands = tuple(self.plans[N].schedule(common.cpu().tolist(), L_top))
        self.sched = Scheduler(specs, budget_bytes, max_cohort)
        self.pending: list = []              # finished cohorts awaiting their event
        self.ticks_in_flight: deque = deque()
        self.t_ref = None                    # (wall time, event) pair for GPU timestamps
        self.next_rid = 0

    def particle_bytes(self, plan, L_top: int) -> int:
        """Device bytes one in-flight particle accounts for: resident
        coefficients (BF16-path and refined), restart state and outputs, plus
        its share of the staging volume and the plan's scratch (expansion
        operands and partial sums, per-band cross-power terms)."""
        C, P, N = plan.C, self.P, plan.N
        V_pad = -(-int(plan.V) // 512) * 512
        resident = 2 * C * 2 * 4 + P * 3 * 8 + 3 * 8 + 8 + 4 + P * 8
        staging = N ** 3 * 4
        scratch = 2 * V_pad * 2 + 2 * 16 * (-(-C // 128) * 128) * 4
        scratch += _band_entries(L_top) * 32 + P * 4 * 8 + 8
        return resident + staging + scratch

    # -- requests --
    def submit(self, req: Request) -> Request:
        if req.template < 0 or req.template >= self.templates[req.box].shape[0]:
            raise ValueError(f"template {req.template} is not resident for {req.box}^3")
        if isinstance(req.volumes, Rows):
            self._check_rows(req, req.volumes)
        if req.arrival is None:
            req.arrival = time.perf_counter()
        if req.rid < 0:
            req.rid = self.next_rid
        self.next_rid = max(self.next_rid, req.rid) + 1
        self.sched.submit(req)
        return req

    def busy(self) -> bool:
        """Requests queued, on the device, or finished but not yet collected."""
        return self.sched.busy() or bool(self.pending)

    # -- one tick --
    def step(self) -> list:
        """Admit, march every live cohort one band, and return the requests
        that completed (their results filled in).  At most two ticks are in
        flight on the device: the call waits for the one before last."""
        torch = self.torch
        if self.t_ref is None:
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(torch.cuda.current_stream(self.dev))
            ev.synchronize()
            self.t_ref = (time.perf_counter(), ev)
        now = time.perf_counter()
        for c in self.sched.admit():
            for r in c.requests:
                r.admitted = now
            self._start(c)
        if not self.sched.live:
            return self._collect()
        for c, band, last in self.sched.plan():
            self._band(c, band, last)
        for c in self.sched.advance():
            self._finish(c)
        marks = []
        for s in self.streams.values():
            ev = torch.cuda.Event()
            ev.record(s)
            marks.append(ev)
        self.ticks_in_flight.append(marks)
        while len(self.ticks_in_flight) > 1:
            for ev in self.ticks_in_flight.popleft():
                ev.synchronize()
        return self._collect()

    def drain(self) -> list:
        """Run ticks until every submitted request has completed."""
        out = []
        while self.sched.busy():
            out += self.step()
        while self.ticks_in_flight:
            for ev in self.ticks_in_flight.popleft():
                ev.synchronize()
        return out + self._collect(block=True)

    def _check_rows(self, r: Request, v: Rows) -> None:
        torch, N = self.torch, r.box
        st, ix = v.stack, v.index
        if (not isinstance(st, torch.Tensor) or not st.is_cuda or st.dtype != torch.float32
                or st.dim() != 4 or tuple(st.shape[1:]) != (N, N, N) or not st.is_contiguous()):
            raise ValueError(f"request {r.rid}: Rows.stack must be a contiguous "
                             f"[n, {N}, {N}, {N}] float32 device tensor")
        if isinstance(ix, torch.Tensor) and ix.is_cuda:
            if ix.dtype != torch.int64 or tuple(ix.shape) != (r.n,):
                raise ValueError(f"request {r.rid}: Rows.index must be [{r.n}] int64")
            return
        h = np.asarray(ix.cpu() if isinstance(ix, torch.Tensor) else ix)
        if h.shape != (r.n,) or h.dtype.kind not in "iu":
            raise ValueError(f"request {r.rid}: Rows.index must hold {r.n} integers")
        if h.size and (h.min() < 0 or h.max() >= st.shape[0]):
            raise ValueError(f"request {r.rid}: Rows.index outside 0..{st.shape[0] - 1}")

    def _cohort_volumes(self, c: Cohort, s):
        """The cohort's volumes on stream s: (stack, int64 row index) when
        every request names rows of one stack (nothing is copied), else one
        [n, N, N, N] tensor (the requests' volumes concatenated)."""
        torch = self.torch
        vols = [r.volumes() if callable(r.volumes) else r.volumes for r in c.requests]
        rows = []
        for r, v in zip(c.requests, vols):
            if isinstance(v, Rows):
                self._check_rows(r, v)
                ix = v.index
                if not (isinstance(ix, torch.Tensor) and ix.is_cuda):
                    # pinned staging, so the copy does not hold the host loop
                    h = np.asarray(ix.cpu() if isinstance(ix, torch.Tensor) else ix,
                                   dtype=np.int64)
                    ix = torch.from_numpy(h).pin_memory().to(self.dev, non_blocking=True)
                v = Rows(v.stack, ix.contiguous())
                v.stack.record_stream(s)
                v.index.record_stream(s)
                rows.append(v)
            else:
                if tuple(v.shape) != (r.n, c.box, c.box, c.box) or v.dtype != torch.float32:
                    raise ValueError(f"request {r.rid}: volumes must be [{r.n}, {c.box}^3] float32")
                v.record_stream(s)
                rows.append(v)
        if all(isinstance(v, Rows) for v in rows):
            st = rows[0].stack
            if all(v.stack.data_ptr() == st.data_ptr() and v.stack.shape == st.shape
                   for v in rows):
                ix = rows[0].index if len(rows) == 1 else torch.cat([v.index for v in rows])
                return st, ix
        mats = [v.stack.index_select(0, v.index) if isinstance(v, Rows) else v for v in rows]
        return (mats[0].contiguous() if len(mats) == 1 else torch.cat(mats)), None

    # -- device work --
    def _start(self, c: Cohort) -> None:
        torch = self.torch
        plan, s = self.plans[c.box], self.streams[c.box]
        # tensors handed in with a request were produced on the caller's
        # stream: the box stream waits for it before reading them, and they
        # are marked as used on the box stream for the caching allocator
        s.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(s):
            v, rows = self._cohort_volumes(c, s)
            starts = [r.starts() if callable(r.starts) else r.starts for r in c.requests]
            for r, st in zip(c.requests, starts):
                if tuple(st.shape) != (r.n, self.P, 3) or st.dtype != torch.float64:
                    raise ValueError(f"request {r.rid}: starts must be [{r.n}, {self.P}, 3] float64")
                st.record_stream(s)
            d = c.dev
            d["a"] = torch.empty((c.n, plan.C, 2), dtype=torch.float32, device=self.dev)
            d["a_bf16"] = torch.empty_like(d["a"])
            if rows is None:
                plan.expand_ex(v, "bf16x3", out=d["a"], coarse=d["a_bf16"], batch_invariant=True)
            else:
                plan.expand_rows(v, rows, "bf16x3", out=d["a"], coarse=d["a_bf16"],
                                 batch_invariant=True)
            del v, rows
            d["state"] = (starts[0].clone() if len(starts) == 1 else torch.cat(starts)).contiguous()
            d["tmpl"] = torch.cat([torch.full((r.n,), r.template, dtype=torch.int32, device=self.dev)
                                   for r in c.requests])
            d["euler"] = torch.empty((c.n, 3), dtype=torch.float64, device=self.dev)
            d["score"] = torch.empty((c.n,), dtype=torch.float64, device=self.dev)
            if self.method == "paper":
                d["all_score"] = torch.empty((c.n, self.P), dtype=torch.float64, device=self.dev)


    def _band(self, c: Cohort, band: int, last: bool) -> None:
        torch = self.torch
        plan, s, d = self.plans[c.box], self.streams[c.box], c.dev
        with torch.cuda.stream(s):
            a = d["a"] if last else d["a_bf16"]
            if self.method == "march":
                plan.align_t(a, self.templates[c.box], d["tmpl"], [band], d["state"], self.steps,
                             *self.step_args, out=(d["euler"], d["score"], d["state"], None),
                             batch_invariant=True)
            elif c.cursor == 0:
                # lowest band: all starts, then the best distinct local maxima
                plan.align_t(a, self.templates[c.box], d["tmpl"], [band], d["state"], self.steps,
                             *self.step_args, out=(d["euler"], d["score"], d["state"], d["all_score"]),
                             batch_invariant=True)
                k = min(self.keep, self.P)
                d["state"], _sc = plan.prune(d["state"], d["all_score"], k, self.min_sep)
                del d["all_score"]
            else:
                plan.align_t(a, self.templates[c.box], d["tmpl"], [band], d["state"],
                             self.steps, *self.step_args,
                             out=(d["euler"], d["score"], d["state"], None), batch_invariant=True,
                             newton_bands=1, newton_steps=self.newton_steps)

    def _finish(self, c: Cohort) -> None:
        torch = self.torch
        s, d = self.streams[c.box], c.dev
        with torch.cuda.stream(s):
            d["euler_h"] = torch.empty((c.n, 3), dtype=torch.float64, pin_memory=True)
            d["score_h"] = torch.empty((c.n,), dtype=torch.float64, pin_memory=True)
            d["euler_h"].copy_(d["euler"], non_blocking=True)
            d["score_h"].copy_(d["score"], non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        d["event"] = ev
        self.pending.append(c)

    def _collect(self, block: bool = False) -> list:
        out, keep = [], []
        wall0, ev0 = self.t_ref if self.t_ref else (None, None)
        for c in self.pending:
            ev = c.dev["event"]
            if block:
                ev.synchronize()
            elif not ev.query():
                keep.append(c)
                continue
            t_done = wall0 + ev0.elapsed_time(ev) / 1e3
            eu, sc = c.dev["euler_h"].numpy(), c.dev["score_h"].numpy()
            o = 0
            for r in c.requests:
                r.euler = eu[o:o + r.n].copy()
                r.score = sc[o:o + r.n].copy()
                r.done = t_done
                o += r.n
                out.append(r)
            c.dev.clear()
        self.pending = keep
        return out

    def close(self) -> None:
        self.torch.cuda.synchronize(self.dev)
        for p in self.plans.values():
            p.close()
        self.plans.clear()


def latency_summary(reqs: Sequence[Request]) -> dict:
    """p50 / p99 / max of completion minus arrival, in milliseconds."""
    lat = np.array([r.done - r.arrival for r in reqs if r.done is not None]) * 1e3
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max())}
