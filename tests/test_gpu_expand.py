"""GPU parity of the expansion (Sec. II-A) against the FP64 oracle.

Bars: per-particle normwise relative error <= 1e-5 (FP32 inputs, FP32 MFMA
with split-K partial sums; the oracle sums the same FP32 samples in FP64),
and for the FP32 path each coefficient within the first-order rounding
bound n 2^-24 sum_v |f psi| (assert_fp32_per_coefficient).
Cases span several 128x128 tiles with ragged particle and coefficient
tails, an odd box (centre voxel at r = 0), B = 0, and the full 64^3, L = 32,
B = 1000 launch shape of the benchmark on sampled particles.
"""

import numpy as np
import pytest

import synth
from gpu_util import cuda_device, normwise, say, to_complex
from oracle import basis, expand

pytestmark = pytest.mark.gpu

TOL = 1e-5


def run_gpu(N, L, vols, with_split=False):
    import torch
    from paper_2509_01180_amd.api import Plan
    dev = cuda_device()
    say(f"expand N={N} L={L} B={len(vols)}")
    plan = Plan(N, L, device=0)
    out = plan.expand(torch.from_numpy(np.ascontiguousarray(vols, dtype=np.float32)).to(dev))
    torch.cuda.synchronize()
    got = to_complex(out)
    split = plan.tuning(max(1, len(vols)))["split_f32"]
    plan.close()
    return (got, split) if with_split else got


def k_steps(N):
    """K-steps of 32 folded voxels of an N^3 plan: one representative per
    mirror orbit inside the ball, the count padded to 512."""
    i = np.arange(N)
    x = (i - (N - 1) / 2) * 2 / N
    half = x[x >= -1e-12]          # one representative per mirror orbit (and the planes)
    X, Y, Z = np.meshgrid(half, half, half, indexing="ij")
    VR = int(((X ** 2 + Y ** 2 + Z ** 2) < 1).sum())
    return -(-VR // 512) * 512 // 32


def fp32_terms(N, nsplit):
    """Rounding steps on the way to one FP32 coefficient: the 8-image fold
    (three levels of additions), the basis entry's FP32 storage, the longest
    run of sequential FP32 accumulations in one split-K slice (the longest
    split's K-steps of 32 folded voxels, the count padded to 512) and the sum
    of the splits."""
    longest = -(-k_steps(N) // nsplit) * 32     # the longest split's K-steps of 32 voxels
    return 3 + 1 + longest + nsplit


def assert_fp32_per_coefficient(got, ref, vols, L, nsplit):
    """Per-coefficient bar of the FP32 path: every rounding is relative to
    the magnitude of the summed terms, so |a_gpu - a| <= n 2^-24 sum_v
    |f(v)| |psi(v)| (first order, n = fp32_terms), for the real and the
    imaginary part separately.  It holds whatever the cancellation in the
    coefficient, so it also catches a single wrong coefficient far below
    the normwise bar."""
    sr, si = split_bf16_scale(vols, L)
    n = fp32_terms(vols.shape[-1], nsplit)
    d = got - ref
    tol = 1.01 * n * 2.0 ** -24
    rr = np.abs(d.real) / np.maximum(sr, 1e-300)
    ri = np.abs(d.imag) / np.maximum(si, 1e-300)
    print(f"per-coefficient error / (2^-24 sum|f psi|): max re {rr.max() / 2.0 ** -24:.1f}, "
          f"im {ri.max() / 2.0 ** -24:.1f}; bound {n}")
    assert np.all(np.abs(d.real) <= tol * sr + 1e-30)
    assert np.all(np.abs(d.imag) <= tol * si + 1e-30)


def test_expand_config1_volumes():
    w = synth.CONFIG1
    vols = np.stack([w.template_volume(), w.particle(0), w.particle(1),
                     w.particle(2, wedge=False, noise=False)])
    ref = expand.expand(vols.astype(np.float64), basis.IndexSet(w.L_max))
    got, split = run_gpu(w.N, w.L_max, vols, with_split=True)
    err = normwise(got, ref)
    print("normwise", err)
    assert np.all(err <= TOL)
    assert_fp32_per_coefficient(got, ref, vols, w.L_max, split)


def test_expand_ragged_tiles():
    # B = 130 spans two particle tiles (128 + 2); C(12) is not a multiple of 128.
    N, L, B = 24, 12, 130
    rng = np.random.default_rng(5)
    vols = rng.standard_normal((B, N, N, N)).astype(np.float32)
    bl = synth.blob_template(rng, 10)
    vols[::7] += 3 * synth.render_blobs(bl, N).astype(np.float32)
    ref = expand.expand(vols.astype(np.float64), basis.IndexSet(L))
    got, split = run_gpu(N, L, vols, with_split=True)
    err = normwise(got, ref)
    assert got.shape == ref.shape
    assert np.all(err <= TOL), err.max()
    assert_fp32_per_coefficient(got, ref, vols, L, split)


def test_expand_odd_box_and_low_bandlimit():
    """Odd boxes put voxels on the three mirror planes (orbits of fewer than
    8 voxels in the folded sum); both the FP32 and the split-BF16 paths."""
    import torch
    from paper_2509_01180_amd.api import Plan
    for N, L in [(17, 6), (9, 0), (15, 9)]:
        rng = np.random.default_rng(N)
        vols = rng.standard_normal((5, N, N, N)).astype(np.float32)
        ref = expand.expand(vols.astype(np.float64), basis.IndexSet(L))
        got, split = run_gpu(N, L, vols, with_split=True)
        assert np.all(normwise(got, ref) <= TOL)
        assert_fp32_per_coefficient(got, ref, vols, L, split)
        plan = Plan(N, L, device=0)
        c3 = plan.expand_ex(torch.from_numpy(vols).to(cuda_device()), "bf16x3")
        torch.cuda.synchronize()
        plan.close()
        # Random volumes cancel heavily, so the split-BF16 bar is per
        # coefficient against sum_v |f psi| (see split_bf16_scale).
        d = to_complex(c3) - ref
        sr, si = split_bf16_scale(vols, L)
        assert np.all(np.abs(d.real) <= 2.0 ** -14 * sr)
        assert np.all(np.abs(d.imag) <= 2.0 ** -14 * si)


def split_bf16_scale(vols, L):
    """sum_v |f(v)| |Re h^3 psi(v)| and the same with Im, per coefficient.

    Split-BF16 (x = hi + lo + r, |lo| <= 2^-9 |x|, |r| <= 2^-18 |x|) keeps
    hi*hi + hi*lo + lo*hi of each product: the dropped parts are at most
    3 * 2^-18 |x y|; FP32 accumulation of K terms adds at most K * 2^-24 of
    the same sum (K <= 500 here).  Both stay below 2^-14 times this scale."""
    N = vols.shape[-1]
    idx = basis.IndexSet(L)
    h, xyz, ball = basis.grid(N)
    P = basis.psi(idx, xyz[ball]) * h ** 3
    F = np.abs(vols.reshape(len(vols), -1)[:, ball.reshape(-1)]).astype(np.float64)
    return F @ np.abs(P.real), F @ np.abs(P.imag)


def test_expand_empty_batch_and_shape_errors():
    import torch
    from paper_2509_01180_amd.api import Plan
    dev = cuda_device()
    plan = Plan(16, 4, device=0)
    out = plan.expand(torch.zeros((0, 16, 16, 16), dtype=torch.float32, device=dev))
    assert out.shape == (0, plan.C, 2)
    with pytest.raises(ValueError):
        plan.expand(torch.zeros((2, 16, 16, 15), dtype=torch.float32, device=dev))
    with pytest.raises(TypeError):
        plan.expand(torch.zeros((2, 16, 16, 16), dtype=torch.float64, device=dev))
    # sizes beyond the ABI's limits are refused before any memory is touched
    from paper_2509_01180_amd._lib import BH_EINVAL, lib
    small = torch.zeros((1, 16, 16, 16), dtype=torch.float32, device=dev)
    coeffs = torch.zeros((1, plan.C, 2), dtype=torch.float32, device=dev)
    assert lib().bh_expand(plan._h, small.data_ptr(), (1 << 21) + 1, coeffs.data_ptr(), None) == BH_EINVAL
    assert lib().bh_expand(plan._h, small.data_ptr(), -1, coeffs.data_ptr(), None) == BH_EINVAL
    plan.close()


def test_expand_deterministic():
    import torch
    from paper_2509_01180_amd.api import Plan
    dev = cuda_device()
    rng = np.random.default_rng(1)
    vols = torch.from_numpy(rng.standard_normal((40, 32, 32, 32)).astype(np.float32)).to(dev)
    plan = Plan(32, 16, device=0)
    a = plan.expand(vols)
    b = plan.expand(vols)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_expand_full_size_sampled():
    """64^3, L = 32, B = 1000 (the benchmark's launch shape); particles at
    sampled positions are workload particles checked against the oracle."""
    w = synth.CONFIG2
    B = w.batch
    sample = [0, 517, 999]
    rng = np.random.default_rng(11)
    vols = (0.1 * rng.standard_normal((B, w.N, w.N, w.N))).astype(np.float32)
    for i in sample:
        vols[i] = w.particle(i)
    ref = expand.expand(vols[sample].astype(np.float64), basis.IndexSet(w.L_max))
    got, split = run_gpu(w.N, w.L_max, vols, with_split=True)
    err = normwise(got[sample], ref)
    print("normwise", err)
    assert np.all(err <= TOL)
    assert np.all(np.isfinite(got))
    assert_fp32_per_coefficient(got[sample], ref, vols[sample], w.L_max, split)


def test_expand_bf16_modes():
    """BF16 expansion (basis and samples rounded to BF16, FP32 accumulation)
    and its split-BF16 refinement against the FP64 oracle.  Bars: BF16 keeps
    ~8 bits per term (2^-9 rounding of each factor), so <= 5e-3 normwise;
    BF16X3 drops only lo*lo and the ~2^-17 split residuals: <= 1e-5."""
    import torch
    from paper_2509_01180_amd.api import Plan
    from paper_2509_01180_amd._lib import BhError
    dev = cuda_device()
    w = synth.CONFIG2
    rng = np.random.default_rng(21)
    B = 200
    vols = (0.1 * rng.standard_normal((B, w.N, w.N, w.N))).astype(np.float32)
    sample = [0, 7, 199]
    for i in sample:
        vols[i] = w.particle(i)
    ref = expand.expand(vols[sample].astype(np.float64), basis.IndexSet(w.L_max))
    say(f"expand bf16 modes N={w.N} L={w.L_max} B={B}")
    plan = Plan(w.N, w.L_max, device=0)
    dv = torch.from_numpy(vols).to(dev)
    c1 = plan.expand_ex(dv, "bf16")
    coarse = torch.empty_like(c1)
    c3 = plan.expand_ex(dv, "bf16x3", coarse=coarse)
    c32 = plan.expand_ex(dv, "fp32")
    torch.cuda.synchronize()
    e1 = normwise(to_complex(c1)[sample], ref)
    e3 = normwise(to_complex(c3)[sample], ref)
    e32 = normwise(to_complex(c32)[sample], ref)
    print(f"normwise error: bf16 {e1}, bf16x3 {e3}, fp32 {e32}")
    assert np.all(e1 <= 5e-3) and np.all(e1 >= 1e-5)     # genuinely BF16
    assert np.all(e3 <= 1e-5)
    # at 200 particles the split-K factor leaves K-step slices of unequal
    # length (split s takes steps [s n / ns, (s + 1) n / ns))
    split = plan.tuning(B)["split_f32"]
    assert k_steps(w.N) % split != 0 and k_steps(w.N) % plan.tuning(B)["split_bf16"] != 0
    assert_fp32_per_coefficient(to_complex(c32)[sample], ref, vols[sample], w.L_max, split)
    np.testing.assert_allclose(coarse.cpu().numpy(), c1.cpu().numpy(), rtol=0, atol=1e-6 * float(c1.abs().max()))
    with pytest.raises(BhError):
        plan.expand_ex(dv, "bf16", coarse=coarse)
    plan.close()


def test_expand_rows_in_place():
    """bh_expand_rows reads vols[rows[b]] from a resident stack: in every
    mode, batch-invariant or not, the same bits as the expansion of the
    gathered copy (rows repeated and out of order, a ragged tile of 131
    particles, a row offset into a wider coefficient array, the coarse
    output); a row outside the stack gives NaN for that particle only and
    BH_EINVAL from the plan's check, the others unchanged."""
    import torch
    from paper_2509_01180_amd.api import Plan
    from paper_2509_01180_amd._lib import BhError
    dev = cuda_device()
    N, L = 20, 8
    rng = np.random.default_rng(33)
    n_vols, B = 57, 131
    stack = torch.from_numpy((rng.standard_normal((n_vols, N, N, N))).astype(np.float32)).to(dev)
    rows_h = rng.integers(0, n_vols, B)
    rows = torch.from_numpy(rows_h).to(dev)
    copy = stack.index_select(0, rows).contiguous()
    say(f"expand_rows N={N} L={L} n_vols={n_vols} B={B}")
    plan = Plan(N, L, device=0)
    C = plan.C
    for mode in ("fp32", "bf16", "bf16x3"):
        for inv in (False, True):
            ref = plan.expand_ex(copy, mode, batch_invariant=inv)
            got = plan.expand_rows(stack, rows, mode, batch_invariant=inv)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (mode, inv)
    wide = torch.full((B, C + 5, 2), 7.0, dtype=torch.float32, device=dev)
    coarse = torch.zeros_like(wide)
    plan.expand_rows(stack, rows, "bf16x3", out=wide, coarse=coarse, batch_invariant=True)
    ref_c = torch.empty((B, C, 2), dtype=torch.float32, device=dev)
    ref = plan.expand_ex(copy, "bf16x3", coarse=ref_c, batch_invariant=True)
    torch.cuda.synchronize()
    assert torch.equal(wide[:, :C], ref) and torch.equal(coarse[:, :C], ref_c)
    assert torch.all(wide[:, C:] == 7.0)
    plan.check()
    # a row outside the stack
    bad = rows.clone()
    bad[5] = n_vols
    bad[9] = -1
    got = plan.expand_rows(stack, bad, "fp32", batch_invariant=True)
    ref = plan.expand_ex(copy, "fp32", batch_invariant=True)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    assert np.all(np.isnan(g[[5, 9], :, 0]))       # (m = 0 imaginary parts are zero by layout)
    keep = np.setdiff1d(np.arange(B), [5, 9])
    np.testing.assert_array_equal(g[keep], ref.cpu().numpy()[keep])
    with pytest.raises(BhError):
        plan.check()
    plan.check()                       # reported once
    with pytest.raises((ValueError, TypeError)):
        plan.expand_rows(stack, rows.to(torch.int32))
    plan.close()
