"""GPU parity of the cross-power and of the Eq. (2) score and Euler gradient.

Both sides receive the same FP32 coefficients; the GPU forms xi in FP64
and evaluates the Wigner small-d recurrence in FP64, so scores and
gradients agree with the oracle far below the 1e-5 bar.  Errors are
measured on the Cauchy-Schwarz scale ||a||_band ||b||_band.
"""

import numpy as np
import pytest

from gpu_util import as_fp32_complex, cuda_device, say, to_pairs
from oracle import basis, expand, score

pytestmark = pytest.mark.gpu

TOL_SCORE = 1e-10      # FP64 on both sides; bar from the method is 1e-5


def random_real_coeffs(idx, B, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((B, idx.size)) + 1j * rng.standard_normal((B, idx.size))
    out = np.stack([expand.real_symmetric(x, idx) for x in c])
    # coefficients decaying with l, like those of smooth volumes
    out *= np.exp(-0.05 * idx.l)[None, :]
    return as_fp32_complex(out)


def random_angles(rng, B, R):
    E = np.stack([rng.uniform(-7, 7, (B, R)), rng.uniform(-1, 4.2, (B, R)),
                  rng.uniform(-7, 7, (B, R))], axis=-1)
    E[:, 0] = [0.3, 0.0, -1.0]          # beta = 0 (gimbal lock)
    if R > 1:
        E[:, 1] = [1.0, np.pi, 2.0]     # beta = pi
    if R > 2:
        E[:, 2] = 0.0                   # identity
    return E


def gpu_tensors(a, b):
    import torch
    dev = cuda_device()
    return (torch.from_numpy(to_pairs(a)).to(dev).contiguous(),
            torch.from_numpy(to_pairs(b)).to(dev).contiguous())


@pytest.mark.parametrize("L", [0, 5, 12])
def test_cross_power_dense(L):
    import torch
    from paper_2509_01180_amd.api import Plan
    Lmax = 12
    idx = basis.IndexSet(Lmax)
    A = random_real_coeffs(idx, 3, 1)
    b = random_real_coeffs(idx, 1, 2)[0]
    da, db = gpu_tensors(A, b)
    say(f"cross_power Lmax={Lmax} L={L} B=3")
    plan = Plan(16, Lmax, device=0)
    xi = plan.cross_power(da, db, L)
    torch.cuda.synchronize()
    got = xi.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    for i in range(3):
        ref = score.cross_power(A[i], b, idx, L)
        flat = np.concatenate([x.reshape(-1) for x in ref])
        scale = np.linalg.norm(A[i]) * np.linalg.norm(b)
        assert np.abs(got[i] - flat).max() <= 1e-13 * scale
    plan.close()


def check_correlate(Lmax, L, B, R, seed, N=16):
    import torch
    from paper_2509_01180_amd.api import Plan
    idx = basis.IndexSet(Lmax)
    A = random_real_coeffs(idx, B, seed)
    b = random_real_coeffs(idx, 1, seed + 100)[0]
    rng = np.random.default_rng(seed + 7)
    E = random_angles(rng, B, R)
    da, db = gpu_tensors(A, b)
    say(f"correlate Lmax={Lmax} L={L} B={B} R={R}")
    plan = Plan(N, Lmax, device=0)
    s, g = plan.correlate(da, db, L, torch.from_numpy(E).to(da.device))
    torch.cuda.synchronize()
    s, g = s.cpu().numpy(), g.cpu().numpy()
    plan.close()
    worst = 0.0
    for i in range(B):
        xi = score.cross_power(A[i], b, idx, L)
        S, G = score.score_grad(xi, E[i])
        scale = max(score.cs_bound(A[i], b, idx, L), 1e-300)
        worst = max(worst, np.abs(s[i] - S).max() / scale, np.abs(g[i] - G).max() / scale)
    print(f"worst error on the CS scale: {worst:.3e}")
    assert worst <= TOL_SCORE


def test_correlate_small_bands():
    check_correlate(16, 16, 3, 100, seed=1)     # two restart chunks, ragged
    check_correlate(16, 7, 2, 5, seed=2)
    check_correlate(4, 0, 2, 1, seed=3)         # L = 0, one rotation


def test_correlate_bandlimit_32():
    check_correlate(32, 32, 3, 64, seed=4)


def test_correlate_high_bandlimit():
    check_correlate(42, 42, 1, 20, seed=5, N=8)


def test_correlate_edge_batches():
    import torch
    from paper_2509_01180_amd.api import Plan
    dev = cuda_device()
    plan = Plan(8, 4, device=0)
    a = torch.zeros((0, plan.C, 2), dtype=torch.float32, device=dev)
    b = torch.zeros((plan.C, 2), dtype=torch.float32, device=dev)
    e = torch.zeros((0, 3, 3), dtype=torch.float64, device=dev)
    s, g = plan.correlate(a, b, 4, e)
    assert s.shape == (0, 3)
    # zero particle -> zero score and gradient
    a1 = torch.zeros((1, plan.C, 2), dtype=torch.float32, device=dev)
    s, g = plan.correlate(a1, b, 4, torch.rand((1, 7, 3), dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    assert torch.count_nonzero(s) == 0 and torch.count_nonzero(g) == 0
    from paper_2509_01180_amd._lib import BhError
    with pytest.raises(BhError):
        plan.correlate(a1, b, 5, torch.zeros((1, 1, 3), dtype=torch.float64, device=dev))
    # coefficient pairs must be 8-byte aligned: a view one float in is refused
    raw = torch.zeros(2 * plan.C + 1, dtype=torch.float32, device=dev)
    shifted = raw[1:].view(1, plan.C, 2)
    assert shifted.data_ptr() % 8 == 4
    with pytest.raises(BhError):
        plan.correlate(shifted, b, 4, torch.zeros((1, 1, 3), dtype=torch.float64, device=dev))
    plan.close()
