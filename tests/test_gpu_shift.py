"""GPU shift search (bh_align_shifts) against the oracle's.

The GPU expands the shifted volumes itself (FP32 MFMA); the oracle expands
the same FP32 samples, shifted, in FP64 and marches from the same starts.
Bars: the same best shift (unless the two best scores tie within 1e-6),
the rotation within 0.5 degrees, the score within 1e-5 (the FP32
expansion's error on the Cauchy-Schwarz scale), and the planted shift and
rotation recovered on noise-free particles.
"""

import numpy as np
import pytest

import synth
from gpu_util import cuda_device, say
from oracle import align as oalign, basis, expand, wigner

pytestmark = pytest.mark.gpu

SHIFTS = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
          (1, 0, -1), (-1, 1, 0)]


def _planted(rng, bl, N, n):
    vols, truth = [], []
    for i in range(n):
        g = synth.quat_to_matrix(synth.haar_quaternions(rng, 1))[0]
        s = SHIFTS[1 + (3 * i) % (len(SHIFTS) - 1)]
        moved = synth.volumes.Blobs(centres=bl.centres @ g.T + np.asarray(s) * (2.0 / N),
                                    amps=bl.amps, sigma=bl.sigma)
        vols.append(synth.render_blobs(moved, N))
        truth.append((s, g))
    return np.stack(vols).astype(np.float32), truth


@pytest.mark.parametrize("N", [20, 17])
def test_align_shifts_vs_oracle(N):
    """N = 17 puts ball voxels on the three mirror planes of the folded
    expansion, where the shifted images of a voxel can coincide."""
    import torch
    from paper_2509_01180_amd.api import Plan
    L = 6
    idx = basis.IndexSet(L)
    rng = np.random.default_rng(21)
    bl = synth.blob_template(rng, 8, radius=0.55)
    vols, truth = _planted(rng, bl, N, 3)
    tv = synth.render_blobs(bl, N).astype(np.float32)
    starts = synth.matrix_to_euler_zyz(synth.quat_to_matrix(
        synth.haar_quaternions(rng, 3 * 16))).reshape(3, 16, 3)
    dev = cuda_device()
    say(f"align_shifts N={N} L={L} B=3 S={len(SHIFTS)} P=16")
    plan = Plan(N, L, device=0)
    b = plan.expand(torch.from_numpy(tv[None]).to(dev))[0].contiguous()
    eu, sc, si = plan.align_shifts(torch.from_numpy(vols).to(dev), b, SHIFTS, (3, 6),
                                   torch.from_numpy(starts).to(dev), 12)
    torch.cuda.synchronize()
    eu, sc, si = eu.cpu().numpy(), sc.cpu().numpy(), si.cpu().numpy()
    plan.close()
    b_ref = expand.expand(tv.astype(np.float64), idx)
    for i in range(3):
        e_ref, s_ref, si_ref = oalign.align_shifts(vols[i], b_ref, idx, SHIFTS, (3, 6),
                                                   starts[i], 12)
        ang = wigner.geodesic_deg(wigner.euler_to_matrix(*eu[i]), wigner.euler_to_matrix(*e_ref))
        print(f"particle {i}: shift {SHIFTS[si[i]]} vs {SHIFTS[si_ref]}, {ang:.3f} deg, "
              f"score {sc[i]:.8g} vs {s_ref:.8g}")
        assert abs(sc[i] - s_ref) <= 1e-5 * abs(s_ref)
        assert si[i] == si_ref
        assert ang <= 0.5
        s_true, g = truth[i]
        assert tuple(SHIFTS[si[i]]) == s_true
        assert wigner.geodesic_deg(wigner.euler_to_matrix(*eu[i]), g.T) < 1.5


def test_align_shifts_errors():
    import torch
    from paper_2509_01180_amd.api import Plan
    from paper_2509_01180_amd._lib import BhError
    dev = cuda_device()
    plan = Plan(16, 4, device=0)
    vols = torch.zeros((1, 16, 16, 16), dtype=torch.float32, device=dev)
    b = torch.zeros((plan.C, 2), dtype=torch.float32, device=dev)
    st = torch.zeros((1, 4, 3), dtype=torch.float64, device=dev)
    with pytest.raises(BhError):
        plan.align_shifts(vols, b, [(17, 0, 0)], (4,), st, 2)        # beyond the box
    with pytest.raises(BhError):
        plan.align_shifts(vols, b, [(0, 0, 0)] * 126, (4,), st, 2)   # too many shifts
    eu, sc, si = plan.align_shifts(vols, b, [(0, 0, 0), (1, 1, 1)], (4,), st, 2)
    torch.cuda.synchronize()
    assert int(si[0]) == 0          # all scores zero: the first shift wins the tie
    plan.close()
