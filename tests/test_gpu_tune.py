"""Autotuning (bh_plan_autotune): the tuned shapes are valid candidates, the
plan reports them, and alignment and expansion after tuning agree with the
results before it (a different wave split only reorders sums)."""

import numpy as np
import pytest

import synth
from gpu_util import cuda_device, normwise, say, to_complex

pytestmark = pytest.mark.gpu


def test_autotune_choices_and_results():
    import torch
    from paper_2509_01180_amd.api import Plan
    dev = cuda_device()
    N, L, B, P = 32, 16, 256, 64
    rng = np.random.default_rng(8)
    bl = synth.blob_template(rng, 20)
    vols = np.stack([synth.add_noise(synth.render_blobs(bl, N, g), 0.5, rng) for g in
                     synth.quat_to_matrix(synth.haar_quaternions(rng, B))]).astype(np.float32)
    starts = torch.from_numpy(synth.matrix_to_euler_zyz(synth.quat_to_matrix(
        synth.haar_quaternions(rng, B * P))).reshape(B, P, 3)).to(dev)
    say(f"autotune N={N} L={L} B={B}")
    plan = Plan(N, L, device=0)
    b = plan.expand(torch.from_numpy(synth.render_blobs(bl, N)[None].astype(np.float32)).to(dev))[0]
    v = torch.from_numpy(vols).to(dev)
    a0 = plan.expand(v)
    e0, s0 = plan.align(a0, b.contiguous(), (8, 16), starts, 10)
    before = plan.tuning(B, (8, 16))
    assert before["waves"] == {8: 0, 16: 0} and before["persistent"] == {8: 0, 16: 0}
    got = plan.autotune(B, (8, 16), restarts=P)
    print("tuned", got)
    assert all(w in (4, 5, 6, 8, 10, 12, 16) for w in got["waves"].values())
    assert 1 <= got["split_f32"] <= 16 and 1 <= got["split_bf16"] <= 16
    a1 = plan.expand(v)
    e1, s1 = plan.align(a1, b.contiguous(), (8, 16), starts, 10)
    torch.cuda.synchronize()
    assert np.all(normwise(to_complex(a1), to_complex(a0)) <= 1e-6)
    s0, s1 = s0.cpu().numpy(), s1.cpu().numpy()
    assert np.max(np.abs(s1 - s0) / np.abs(s0)) <= 1e-6
    plan.close()


def test_persistent_launches_match():
    """Persistent workgroups (fewer than the particles, looping) give the
    same bits as one workgroup per particle with the same wave count."""
    import torch
    from paper_2509_01180_amd.api import Plan
    from paper_2509_01180_amd._lib import BhError
    dev = cuda_device()
    N, L, B, P = 20, 12, 1200, 64
    rng = np.random.default_rng(9)
    bl = synth.blob_template(rng, 12)
    vols = np.stack([synth.render_blobs(bl, N, g) for g in
                     synth.quat_to_matrix(synth.haar_quaternions(rng, B))]).astype(np.float32)
    starts = torch.from_numpy(synth.matrix_to_euler_zyz(synth.quat_to_matrix(
        synth.haar_quaternions(rng, B * P))).reshape(B, P, 3)).to(dev)
    say(f"persistent march N={N} L={L} B={B}")
    plan = Plan(N, L, device=0)
    b = plan.expand(torch.from_numpy(synth.render_blobs(bl, N)[None].astype(np.float32)).to(dev))[0]
    a = plan.expand(torch.from_numpy(vols).to(dev))
    for Lb in (6, 12):
        plan.set_tuning(Lb, 12, False)
    ref = plan.align(a, b.contiguous(), (6, 12), starts, 5, return_all=True)
    for Lb in (6, 12):
        plan.set_tuning(Lb, 12, True)
    got = plan.align(a, b.contiguous(), (6, 12), starts, 5, return_all=True)
    torch.cuda.synchronize()
    for x, y in zip(ref, got):
        assert torch.equal(x, y)
    assert plan.tuning(B, (6, 12))["persistent"] == {6: 1, 12: 1}
    with pytest.raises(BhError):
        plan.set_tuning(2, 12, False)      # more waves than p-groups at L = 2
    with pytest.raises(BhError):
        plan.set_tuning(6, 7, False)
    plan.close()


def test_march_split_over_two_streams_same_bits():
    """A march of 512 or more particles runs as two halves on two streams;
    every particle's result (best and all restarts) is the same bits as with
    the split off, for one template and for a template table (batch-invariant
    form), and the profiler's busy time of the ascent launches is at most
    the sum of their durations."""
    import torch
    from paper_2509_01180_amd.api import Plan
    dev = cuda_device()
    N, L, B, P = 16, 8, 600, 64
    rng = np.random.default_rng(21)
    bl = synth.blob_template(rng, 10)
    vols = np.stack([synth.add_noise(synth.render_blobs(bl, N, g), 0.5, rng) for g in
                     synth.quat_to_matrix(synth.haar_quaternions(rng, B))]).astype(np.float32)
    starts = torch.from_numpy(synth.matrix_to_euler_zyz(synth.quat_to_matrix(
        synth.haar_quaternions(rng, B * P))).reshape(B, P, 3)).to(dev)
    say(f"two-stream march N={N} L={L} B={B}")
    plan = Plan(N, L, device=0)
    b = plan.expand(torch.from_numpy(synth.render_blobs(bl, N)[None].astype(np.float32)).to(dev))
    a = plan.expand(torch.from_numpy(vols).to(dev))
    tabs = torch.cat([b, 0.5 * b, b.flip(1)]).contiguous()
    ti = torch.from_numpy(rng.integers(0, 3, B).astype(np.int32)).to(dev)
    res = {}
    for streams in (1, 2):
        plan.set_march_streams(streams)
        plan.profile(True)
        r1 = plan.align(a, b[0].contiguous(), (4, 8), starts, 6, return_all=True)
        r2 = plan.align_t(a, tabs, ti, (4, 8), starts, 6, return_all=True, batch_invariant=True)
        torch.cuda.synchronize()
        plan.profile(False)
        n, ms, _w = plan.profile_read("march_L*")
        busy = plan.profile_busy("march_L*")
        assert 0.0 < busy <= ms * (1 + 1e-6)
        assert n == (4 if streams == 1 else 8)
        res[streams] = [x.cpu() for x in r1] + [x.cpu() for x in r2]
    for x, y in zip(res[1], res[2]):
        assert torch.equal(x, y)
    assert np.all(np.isfinite(res[2][1].numpy()))
    with pytest.raises(Exception):
        plan.set_march_streams(3)
    plan.close()
