"""Python binding of the C ABI (include/bh.h) on torch tensors.

Argument marshalling only: shapes and dtypes are checked, device pointers
and the current HIP stream are handed to libbh, and every computation runs
in the library's kernels.  Torch provides device memory and streams.
"""

from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from ._lib import BH_EXPAND_BATCH_INVARIANT, AlignOpts, check, lib

__all__ = ["Plan", "index_size", "index_table", "radial_table", "ball_voxels",
           "dense_xi_size"]


def index_size(L: int) -> int:
    """C(L): number of complex coefficients of band L."""
    return check(lib().bh_index_size(int(L)), "bh_index_size")


def index_table(L: int):
    """Per-coefficient (l, k, m, lambda_lk) arrays of band L (host)."""
    n = index_size(L)
    l = np.zeros(n, np.int32)
    k = np.zeros(n, np.int32)
    m = np.zeros(n, np.int32)
    lam = np.zeros(n, np.float64)
    check(lib().bh_index_table(int(L), _i32(l), _i32(k), _i32(m), _f64(lam)), "bh_index_table")
    return l, k, m, lam


def radial_table(L: int):
    """Per-radial-entry (l, k, lambda_lk, c_lk) arrays of band L (host)."""
    n = check(lib().bh_radial_count(int(L)), "bh_radial_count")
    l = np.zeros(n, np.int32)
    k = np.zeros(n, np.int32)
    lam = np.zeros(n, np.float64)
    c = np.zeros(n, np.float64)
    check(lib().bh_radial_table(int(L), _i32(l), _i32(k), _f64(lam), _f64(c)), "bh_radial_table")
    return l, k, lam, c


def ball_voxels(N: int) -> int:
    return check(lib().bh_ball_voxels(int(N)), "bh_ball_voxels")


def dense_xi_size(L: int) -> int:
    """E(L) = sum_{l<=L} (2l+1)^2."""
    return (L + 1) * (4 * (L + 1) ** 2 - 1) // 3


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, shape, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Plan:
    """A basis plan for box edge N and bandlimit L_max on one GPU."""

    def __init__(self, N: int, L_max: int, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.N, self.L_max, self.device = int(N), int(L_max), int(device)
        h = ctypes.c_void_p()
        check(lib().bh_plan_create(self.N, self.L_max, self.device, ctypes.byref(h)),
              "bh_plan_create")
        self._h = h
        self.C = self.num_coeffs(self.L_max)
        self.V = ball_voxels(self.N)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().bh_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def check(self) -> None:
        """Synchronise the current stream and raise BhError (BH_EINVAL) if a
        kernel of this plan met a template index outside its table or a
        volume row outside its stack since the last check (see
        bh_plan_check)."""
        check(lib().bh_plan_check(self._h, _stream()), "bh_plan_check")

    def num_coeffs(self, L: int) -> int:
        return check(lib().bh_plan_num_coeffs(self._h, int(L)), "bh_plan_num_coeffs")

    # ------------------------------------------------------- autotuning --
    def autotune(self, B: int, bands: Sequence[int] = (), restarts: int = 64,
                 what: Sequence[str] = ("march", "expand", "expand_bf16")) -> dict:
        """Time the candidate launch shapes on this GPU for batch size B and
        keep the fastest in the plan (see bh_plan_autotune); returns the
        choices now in effect for each band and for B."""
        from ._lib import BH_TUNE_EXPAND, BH_TUNE_EXPAND_BF16, BH_TUNE_MARCH
        flags = {"march": BH_TUNE_MARCH, "expand": BH_TUNE_EXPAND,
                 "expand_bf16": BH_TUNE_EXPAND_BF16}
        code = 0
        for w in what:
            code |= flags[w]
        bl = (ctypes.c_int32 * max(1, len(bands)))(*[int(x) for x in bands])
        check(lib().bh_plan_autotune(self._h, int(B), int(restarts), bl, len(bands), code,
                                     _stream()), "bh_plan_autotune")
        return self.tuning(B, bands)

    def set_tuning(self, L: int, waves: int = 0, persistent: bool = False) -> None:
        """Pin the ascent kernel's wave count / persistence for band L."""
        check(lib().bh_plan_set_tuning(self._h, int(L), int(waves), int(bool(persistent))),
              "bh_plan_set_tuning")

    def tuning(self, B: int, bands: Sequence[int] = ()) -> dict:
        """{"waves": {L: tuned wave count or 0}, "persistent": {L: 0/1},
        "split_f32": s, "split_bf16": s}."""
        w, ps, s32, s16 = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        out = {"waves": {}, "persistent": {}}
        for L in bands:
            check(lib().bh_plan_tuning(self._h, int(L), int(B), ctypes.byref(w), ctypes.byref(ps),
                                       ctypes.byref(s32), ctypes.byref(s16)), "bh_plan_tuning")
            out["waves"][int(L)] = w.value
            out["persistent"][int(L)] = ps.value
        check(lib().bh_plan_tuning(self._h, 0, int(B), ctypes.byref(w), ctypes.byref(ps),
                                   ctypes.byref(s32), ctypes.byref(s16)), "bh_plan_tuning")
        out["split_f32"], out["split_bf16"] = s32.value, s16.value
        return out

    # ------------------------------------------------------- profiling --
    def profile(self, enable: bool = True) -> None:
        """Start (clearing earlier records) or stop per-kernel event timing."""
        check(lib().bh_profile_enable(self._h, 1 if enable else 0), "bh_profile_enable")

    def profile_read(self, name: str):
        """(launches, total_ms, work_units) of the recorded kernels named `name`
        (a trailing '*' matches a prefix)."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        w = ctypes.c_int64()
        check(lib().bh_profile_read(self._h, name.encode(), ctypes.byref(n), ctypes.byref(ms),
                                    ctypes.byref(w)), "bh_profile_read")
        return n.value, ms.value, w.value

    def profile_busy(self, name: str) -> float:
        """Milliseconds during which a recorded kernel named `name` was running
        (the union over launches and streams; see bh_profile_busy)."""
        ms = ctypes.c_double()
        check(lib().bh_profile_busy(self._h, name.encode(), ctypes.byref(ms)), "bh_profile_busy")
        return ms.value

    def set_march_streams(self, streams: int) -> None:
        """1: never split a march over two streams; 2 (default): split
        eligible batches (see bh_plan_set_march_streams)."""
        check(lib().bh_plan_set_march_streams(self._h, int(streams)), "bh_plan_set_march_streams")

    # ----------------------------------------------------------- calls --
    def expand(self, vols: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """vols [B, N, N, N] float32 -> coefficients [B, C(L_max), 2] float32."""
        B = vols.shape[0]
        _dev(vols, torch.float32, (B, self.N, self.N, self.N), "vols")
        if out is None:
            out = torch.empty((B, self.C, 2), dtype=torch.float32, device=vols.device)
        _dev(out, torch.float32, (B, self.C, 2), "out")
        check(lib().bh_expand(self._h, _ptr(vols), B, _ptr(out), _stream()), "bh_expand")
        return out

    def expand_ex(self, vols: torch.Tensor, mode: str = "fp32", out: torch.Tensor | None = None,
                  coarse: torch.Tensor | None = None,
                  batch_invariant: bool = False) -> torch.Tensor:
        """Expansion in mode "fp32", "bf16" or "bf16x3" (see bh_expand_ex).

        With mode "bf16x3" and a `coarse` tensor [B, C, 2], the BF16 (hi*hi)
        result is written there too.  With batch_invariant, each particle's
        coefficients are the same bits whatever batch it is expanded in.
        """
        modes = {"fp32": 0, "bf16": 1, "bf16x3": 2}
        code = modes[mode] | (BH_EXPAND_BATCH_INVARIANT if batch_invariant else 0)
        B = vols.shape[0]
        _dev(vols, torch.float32, (B, self.N, self.N, self.N), "vols")
        if out is None:
            out = torch.empty((B, self.C, 2), dtype=torch.float32, device=vols.device)
        _dev(out, torch.float32, (B, self.C, 2), "out")
        if coarse is not None:
            _dev(coarse, torch.float32, (B, self.C, 2), "coarse")
        check(lib().bh_expand_ex(self._h, _ptr(vols), B, code, _ptr(out), _ptr(coarse),
                                 _stream()), "bh_expand_ex")
        return out

    def expand_noalloc(self, vols: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """bh_expand_noalloc: the batch-invariant FP32 expansion with the
        library's static device scratch (no device allocation in the call).
        `out` [B, C(L_max), 2] float32 is supplied by the caller."""
        B = vols.shape[0]
        _dev(vols, torch.float32, (B, self.N, self.N, self.N), "vols")
        _dev(out, torch.float32, (B, self.C, 2), "out")
        check(lib().bh_expand_noalloc(self._h, _ptr(vols), B, _ptr(out), _stream()),
              "bh_expand_noalloc")
        return out

    def noalloc_batch(self) -> int:
        """Particles per pass of expand_noalloc (0: the plan does not fit)."""
        return check(lib().bh_expand_noalloc_batch(self._h), "bh_expand_noalloc_batch")

    def expand_into(self, vols: torch.Tensor, out: torch.Tensor, mode: str = "fp32",
                    coarse: torch.Tensor | None = None, batch_invariant: bool = False):
        """Expansion into rows of a wider coefficient array: out [B, ldc, 2]
        float32 with ldc >= C (the first C entries of each row are written)."""
        modes = {"fp32": 0, "bf16": 1, "bf16x3": 2}
        code = modes[mode] | (BH_EXPAND_BATCH_INVARIANT if batch_invariant else 0)
        B = vols.shape[0]
        _dev(vols, torch.float32, (B, self.N, self.N, self.N), "vols")
        ldc = out.shape[1]
        _dev(out, torch.float32, (B, ldc, 2), "out")
        if coarse is not None:
            _dev(coarse, torch.float32, (B, ldc, 2), "coarse")
        check(lib().bh_expand_into(self._h, _ptr(vols), B, code, _ptr(out), ldc, _ptr(coarse),
                                   _stream()), "bh_expand_into")
        return out

    def expand_rows(self, vols: torch.Tensor, rows: torch.Tensor, mode: str = "fp32",
                    out: torch.Tensor | None = None, coarse: torch.Tensor | None = None,
                    batch_invariant: bool = False) -> torch.Tensor:
        """Expansion of the volumes vols[rows[b]] read in place from a
        resident stack vols [n, N, N, N] float32 (see bh_expand_rows); rows
        is an int64 device tensor [B].  out (and coarse, mode "bf16x3")
        [B, ldc, 2] float32 with ldc >= C; the same bits as expand_into on
        vols[rows]."""
        modes = {"fp32": 0, "bf16": 1, "bf16x3": 2}
        code = modes[mode] | (BH_EXPAND_BATCH_INVARIANT if batch_invariant else 0)
        n = vols.shape[0]
        _dev(vols, torch.float32, (n, self.N, self.N, self.N), "vols")
        B = rows.shape[0] if rows.dim() == 1 else -1
        _dev(rows, torch.int64, (B,), "rows")
        if out is None:
            out = torch.empty((B, self.C, 2), dtype=torch.float32, device=vols.device)
        ldc = out.shape[1]
        _dev(out, torch.float32, (B, ldc, 2), "out")
        if coarse is not None:
            _dev(coarse, torch.float32, (B, ldc, 2), "coarse")
        check(lib().bh_expand_rows(self._h, _ptr(vols), n, _ptr(rows), B, code, _ptr(out), ldc,
                                   _ptr(coarse), _stream()), "bh_expand_rows")
        return out

    def align_uneven(self, a: torch.Tensor, Lp, templates: torch.Tensor,
                     tmpl_idx: torch.Tensor | None, bands: Sequence[int], starts: torch.Tensor,
                     steps: int, step_init: float = 1.0, step_grow: float = 1.25,
                     step_shrink: float = 0.5, return_all: bool = False,
                     batch_invariant: bool = False, newton_bands: int = 0, newton_steps: int = 0,
                     keep: int = 0, min_sep: float = 0.0, out: tuple | None = None):
        """Particles of several bandlimits in one march (see bh_align_uneven):
        a [B, lda, 2], Lp (B ints, non-increasing), templates [T, ldt, 2].
        out: optional (euler, score, all_euler, all_score) buffers to fill."""
        import numpy as np
        B, lda = a.shape[0], a.shape[1]
        T, ldt = templates.shape[0], templates.shape[1]
        P = starts.shape[1]
        _dev(a, torch.float32, (B, lda, 2), "a")
        _dev(templates, torch.float32, (T, ldt, 2), "templates")
        _dev(starts, torch.float64, (B, P, 3), "starts")
        if tmpl_idx is not None:
            _dev(tmpl_idx, torch.int32, (B,), "tmpl_idx")
        lp = np.ascontiguousarray(np.asarray(Lp, dtype=np.int32))
        if lp.shape != (B,):
            raise ValueError("Lp must hold one bandlimit per particle")
        bl = (ctypes.c_int32 * len(bands))(*[int(x) for x in bands])
        o = AlignOpts(ctypes.cast(bl, ctypes.POINTER(ctypes.c_int32)), len(bands), int(steps), P,
                      float(step_init), float(step_grow), float(step_shrink),
                      int(bool(batch_invariant)), int(newton_bands), int(newton_steps),
                      int(keep), float(min_sep))
        Po = keep if 0 < keep < P else P
        if out is None:
            eu = torch.empty((B, 3), dtype=torch.float64, device=a.device)
            sc = torch.empty((B,), dtype=torch.float64, device=a.device)
            ae = torch.empty((B, Po, 3), dtype=torch.float64, device=a.device) if return_all else None
            asc = torch.empty((B, Po), dtype=torch.float64, device=a.device) if return_all else None
        else:
            eu, sc, ae, asc = out
            _dev(eu, torch.float64, (B, 3), "euler_out")
            _dev(sc, torch.float64, (B,), "score_out")
            if ae is not None:
                _dev(ae, torch.float64, (B, Po, 3), "all_euler")
            if asc is not None:
                _dev(asc, torch.float64, (B, Po), "all_score")
        check(lib().bh_align_uneven(self._h, _ptr(a), lda, lp.ctypes.data_as(ctypes.c_void_p),
                                    _ptr(templates), ldt, T, _ptr(tmpl_idx), B, ctypes.byref(o),
                                    _ptr(starts), _ptr(eu), _ptr(sc), _ptr(ae), _ptr(asc),
                                    _stream()), "bh_align_uneven")
        if return_all:
            return eu, sc, ae, asc
        return eu, sc

    def cross_power(self, a: torch.Tensor, b: torch.Tensor, L: int) -> torch.Tensor:
        """xi [B, E(L), 2] float64 (blocks l, row-major [m][n])."""
        B = a.shape[0]
        _dev(a, torch.float32, (B, self.C, 2), "a")
        _dev(b, torch.float32, (self.C, 2), "b")
        out = torch.empty((B, dense_xi_size(L), 2), dtype=torch.float64, device=a.device)
        check(lib().bh_cross_power(self._h, _ptr(a), _ptr(b), B, int(L), _ptr(out), _stream()),
              "bh_cross_power")
        return out

    def correlate(self, a: torch.Tensor, b: torch.Tensor, L: int, euler: torch.Tensor,
                  grad: bool = True):
        """Score [B, R] and Euler gradient [B, R, 3] (float64) at euler [B, R, 3]."""
        B = a.shape[0]
        R = euler.shape[1]
        _dev(a, torch.float32, (B, self.C, 2), "a")
        _dev(b, torch.float32, (self.C, 2), "b")
        _dev(euler, torch.float64, (B, R, 3), "euler")
        score = torch.empty((B, R), dtype=torch.float64, device=a.device)
        g = torch.empty((B, R, 3), dtype=torch.float64, device=a.device) if grad else None
        check(lib().bh_correlate(self._h, _ptr(a), _ptr(b), B, int(L), _ptr(euler), R,
                                 _ptr(score), _ptr(g), _stream()), "bh_correlate")
        return score, g

    def correlate_hess(self, a: torch.Tensor, b: torch.Tensor, L: int, euler: torch.Tensor):
        """Score [B, R], gradient [B, R, 3] and Hessian [B, R, 3, 3] (float64)."""
        B = a.shape[0]
        R = euler.shape[1]
        _dev(a, torch.float32, (B, self.C, 2), "a")
        _dev(b, torch.float32, (self.C, 2), "b")
        _dev(euler, torch.float64, (B, R, 3), "euler")
        score = torch.empty((B, R), dtype=torch.float64, device=a.device)
        g = torch.empty((B, R, 3), dtype=torch.float64, device=a.device)
        h6 = torch.empty((B, R, 6), dtype=torch.float64, device=a.device)
        check(lib().bh_correlate_hess(self._h, _ptr(a), _ptr(b), B, int(L), _ptr(euler), R,
                                      _ptr(score), _ptr(g), _ptr(h6), _stream()),
              "bh_correlate_hess")
        idx = torch.tensor([[0, 1, 2], [1, 3, 4], [2, 4, 5]], device=a.device)
        return score, g, h6[:, :, idx]

    def prune(self, euler: torch.Tensor, score: torch.Tensor, K: int, min_sep: float,
              out: tuple | None = None):
        """K candidates per particle from euler [B, P, 3] / score [B, P]
        (see bh_prune_candidates): (euler [B, K, 3], score [B, K])."""
        B, P = score.shape
        _dev(euler, torch.float64, (B, P, 3), "euler")
        _dev(score, torch.float64, (B, P), "score")
        if out is None:
            out = (torch.empty((B, K, 3), dtype=torch.float64, device=euler.device),
                   torch.empty((B, K), dtype=torch.float64, device=euler.device))
        eo, so = out
        _dev(eo, torch.float64, (B, K, 3), "euler_out")
        _dev(so, torch.float64, (B, K), "score_out")
        check(lib().bh_prune_candidates(self._h, _ptr(euler), _ptr(score), B, P, int(K),
                                        float(min_sep), _ptr(eo), _ptr(so), _stream()),
              "bh_prune_candidates")
        return eo, so

    def degree_energy(self, a: torch.Tensor, b: torch.Tensor, L: int) -> torch.Tensor:
        """||xi^l||_F^2 of the band-L cross-power, [B, L+1] float64."""
        B = a.shape[0]
        _dev(a, torch.float32, (B, self.C, 2), "a")
        _dev(b, torch.float32, (self.C, 2), "b")
        out = torch.empty((B, int(L) + 1), dtype=torch.float64, device=a.device)
        check(lib().bh_degree_energy(self._h, _ptr(a), _ptr(b), B, int(L), _ptr(out), _stream()),
              "bh_degree_energy")
        return out

    def select_bands(self, a: torch.Tensor, templates: torch.Tensor,
                     tmpl_idx: torch.Tensor | None, L_top: int, thresholds: Sequence[float],
                     ratio: bool = False, out: tuple | None = None):
        """Energy-ratio band selection (see bh_select_bands).

        templates: [T, C, 2] float32 (or [C, 2] for one template); tmpl_idx:
        [B] int32 (None if T == 1).  Returns (bands [B, n_tau] int32, common
        [n_tau] int32, ratio [B, L_top + 1] float64 or None), all on the
        device; out: optional (bands, common) buffers to fill."""
        import numpy as np
        B = a.shape[0]
        if templates.dim() == 2:
            templates = templates.unsqueeze(0)
        T = templates.shape[0]
        _dev(a, torch.float32, (B, self.C, 2), "a")
        _dev(templates, torch.float32, (T, self.C, 2), "templates")
        if tmpl_idx is not None:
            _dev(tmpl_idx, torch.int32, (B,), "tmpl_idx")
        th = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float64).reshape(-1))
        n = len(th)
        if out is None:
            bands = torch.empty((B, n), dtype=torch.int32, device=a.device)
            common = torch.empty((n,), dtype=torch.int32, device=a.device)
        else:
            bands, common = out
            _dev(bands, torch.int32, (B, n), "bands")
            _dev(common, torch.int32, (n,), "common")
        r = (torch.empty((B, int(L_top) + 1), dtype=torch.float64, device=a.device)
             if ratio else None)
        check(lib().bh_select_bands(self._h, _ptr(a), _ptr(templates), T, _ptr(tmpl_idx), B,
                                    int(L_top), _f64(th), n, _ptr(bands), _ptr(common), _ptr(r),
                                    _stream()), "bh_select_bands")
        return bands, common, r

    @staticmethod
    def schedule(common, L_top: int) -> list:
        """March schedule from the batch choices of select_bands: the
        distinct choices above 0, increasing, then L_top."""
        vals = sorted({int(x) for x in common} - {0} - {int(L_top)})
        return vals + [int(L_top)]

    def align(self, a: torch.Tensor, b: torch.Tensor, bands: Sequence[int], starts: torch.Tensor,
              steps: int, step_init: float = 1.0, step_grow: float = 1.25,
              step_shrink: float = 0.5, return_all: bool = False,
              batch_invariant: bool = False, newton_bands: int = 0, newton_steps: int = 0,
              keep: int = 0, min_sep: float = 0.0):
        """Best rotation per particle: (euler [B, 3], score [B]) float64.

        With return_all, also the final point [B, P', 3] and score [B, P'] of
        every restart (P' = keep when candidates are pruned).  With
        batch_invariant, each particle's result is independent of the batch
        it is aligned in.  newton_bands / newton_steps / keep / min_sep: see
        bh_align_opts (Newton bands, candidates after the first band).
        """
        B = a.shape[0]
        P = starts.shape[1]
        _dev(a, torch.float32, (B, self.C, 2), "a")
        _dev(b, torch.float32, (self.C, 2), "b")
        _dev(starts, torch.float64, (B, P, 3), "starts")
        bl = (ctypes.c_int32 * len(bands))(*[int(x) for x in bands])
        o = AlignOpts(ctypes.cast(bl, ctypes.POINTER(ctypes.c_int32)), len(bands), int(steps), P,
                      float(step_init), float(step_grow), float(step_shrink),
                      int(bool(batch_invariant)), int(newton_bands), int(newton_steps),
                      int(keep), float(min_sep))
        eu = torch.empty((B, 3), dtype=torch.float64, device=a.device)
        sc = torch.empty((B,), dtype=torch.float64, device=a.device)
        Po = keep if 0 < keep < P else P
        ae = torch.empty((B, Po, 3), dtype=torch.float64, device=a.device) if return_all else None
        asc = torch.empty((B, Po), dtype=torch.float64, device=a.device) if return_all else None
        check(lib().bh_align(self._h, _ptr(a), _ptr(b), B, ctypes.byref(o), _ptr(starts),
                             _ptr(eu), _ptr(sc), _ptr(ae), _ptr(asc), _stream()), "bh_align")
        if return_all:
            return eu, sc, ae, asc
        return eu, sc

    def align_shifts(self, vols: torch.Tensor, b: torch.Tensor, shifts, bands: Sequence[int],
                     starts: torch.Tensor, steps: int, step_init: float = 1.0,
                     step_grow: float = 1.25, step_shrink: float = 0.5, newton_bands: int = 0,
                     newton_steps: int = 0, keep: int = 0, min_sep: float = 0.0):
        """Shift search: (euler [B, 3], score [B], shift index [B]) over the
        integer voxel shifts (sequence of (dx, dy, dz)); see bh_align_shifts."""
        import numpy as np
        B = vols.shape[0]
        P = starts.shape[1]
        _dev(vols, torch.float32, (B, self.N, self.N, self.N), "vols")
        _dev(b, torch.float32, (self.C, 2), "b")
        _dev(starts, torch.float64, (B, P, 3), "starts")
        sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.int32).reshape(-1, 3))
        bl = (ctypes.c_int32 * len(bands))(*[int(x) for x in bands])
        o = AlignOpts(ctypes.cast(bl, ctypes.POINTER(ctypes.c_int32)), len(bands), int(steps), P,
                      float(step_init), float(step_grow), float(step_shrink), 0,
                      int(newton_bands), int(newton_steps), int(keep), float(min_sep))
        eu = torch.empty((B, 3), dtype=torch.float64, device=vols.device)
        sc = torch.empty((B,), dtype=torch.float64, device=vols.device)
        si = torch.empty((B,), dtype=torch.int32, device=vols.device)
        check(lib().bh_align_shifts(self._h, _ptr(vols), B, sh.ctypes.data_as(ctypes.c_void_p),
                                    len(sh), _ptr(b), ctypes.byref(o), _ptr(starts), _ptr(eu),
                                    _ptr(sc), _ptr(si), _stream()), "bh_align_shifts")
        return eu, sc, si

    def align_t(self, a: torch.Tensor, templates: torch.Tensor, tmpl_idx: torch.Tensor | None,
                bands: Sequence[int], starts: torch.Tensor, steps: int, step_init: float = 1.0,
                step_grow: float = 1.25, step_shrink: float = 0.5, return_all: bool = False,
                out: tuple | None = None, batch_invariant: bool = False, newton_bands: int = 0,
                newton_steps: int = 0, keep: int = 0, min_sep: float = 0.0):
        """As align, with particle i matched against templates[tmpl_idx[i]].

        templates: [T, C, 2] float32; tmpl_idx: [B] int32 (None if T == 1).
        out: optional (euler, score, all_euler, all_score) buffers to fill.
        """
        B = a.shape[0]
        P = starts.shape[1]
        T = templates.shape[0]
        _dev(a, torch.float32, (B, self.C, 2), "a")
        _dev(templates, torch.float32, (T, self.C, 2), "templates")
        _dev(starts, torch.float64, (B, P, 3), "starts")
        if tmpl_idx is not None:
            _dev(tmpl_idx, torch.int32, (B,), "tmpl_idx")
        Po = keep if 0 < keep < P else P
        bl = (ctypes.c_int32 * len(bands))(*[int(x) for x in bands])
        o = AlignOpts(ctypes.cast(bl, ctypes.POINTER(ctypes.c_int32)), len(bands), int(steps), P,
                      float(step_init), float(step_grow), float(step_shrink),
                      int(bool(batch_invariant)), int(newton_bands), int(newton_steps),
                      int(keep), float(min_sep))
        if out is None:
            eu = torch.empty((B, 3), dtype=torch.float64, device=a.device)
            sc = torch.empty((B,), dtype=torch.float64, device=a.device)
            ae = torch.empty((B, Po, 3), dtype=torch.float64, device=a.device) if return_all else None
            asc = torch.empty((B, Po), dtype=torch.float64, device=a.device) if return_all else None
        else:
            eu, sc, ae, asc = out
            _dev(eu, torch.float64, (B, 3), "euler_out")
            _dev(sc, torch.float64, (B,), "score_out")
            if ae is not None:
                _dev(ae, torch.float64, (B, Po, 3), "all_euler")
            if asc is not None:
                _dev(asc, torch.float64, (B, Po), "all_score")
        check(lib().bh_align_t(self._h, _ptr(a), _ptr(templates), T, _ptr(tmpl_idx), B,
                               ctypes.byref(o), _ptr(starts), _ptr(eu), _ptr(sc), _ptr(ae),
                               _ptr(asc), _stream()), "bh_align_t")
        if return_all:
            return eu, sc, ae, asc
        return eu, sc
