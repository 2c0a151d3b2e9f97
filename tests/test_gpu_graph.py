"""HIP-graph capture of a marching call (GraphedAlign).

Each replay must give bit-for-bit the eager call's result, also with other
eager work and synchronisations between the replays and with the inputs
refilled in place; a small batch is timed eager vs replayed (printed).
"""

import time

import numpy as np
import pytest

import synth
from gpu_util import cuda_device, say

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager():
    import torch
    from paper_2509_01180_amd.api import Plan
    from paper_2509_01180_amd.graphs import GraphedAlign
    dev = cuda_device()
    N, L, B, P = 24, 12, 6, 32
    rng = np.random.default_rng(5)
    bl = synth.blob_template(rng, 12)
    vols = np.stack([synth.add_noise(synth.render_blobs(bl, N, g), 1.0, rng) for g in
                     synth.quat_to_matrix(synth.haar_quaternions(rng, 2 * B))]).astype(np.float32)
    starts = synth.matrix_to_euler_zyz(synth.quat_to_matrix(
        synth.haar_quaternions(rng, 2 * B * P))).reshape(2 * B, P, 3)
    say(f"graph capture N={N} L={L} B={B} P={P}")
    plan = Plan(N, L, device=0)
    tmpl = plan.expand(torch.from_numpy(synth.render_blobs(bl, N)[None].astype(np.float32)).to(dev))
    A = plan.expand(torch.from_numpy(vols).to(dev))
    S = torch.from_numpy(starts).to(dev)
    bands = (4, 8, 12)
    a = A[:B].clone()
    st = S[:B].clone()
    g = GraphedAlign(plan, a, tmpl, None, bands, st, 10)
    ref = [plan.align_t(A[k * B:(k + 1) * B].contiguous(), tmpl, None, bands,
                        S[k * B:(k + 1) * B].contiguous(), 10) for k in range(2)]
    torch.cuda.synchronize()
    for rep in range(4):
        k = rep % 2
        a.copy_(A[k * B:(k + 1) * B])
        st.copy_(S[k * B:(k + 1) * B])
        eu, sc = g.replay()
        other = plan.align_t(A[B:].contiguous(), tmpl, None, (4,), S[B:].contiguous(), 3)  # eager work
        torch.cuda.synchronize()
        assert torch.equal(eu, ref[k][0]) and torch.equal(sc, ref[k][1]), rep
        assert torch.all(torch.isfinite(other[1]))
    # launch cost: replay vs eager on the same small batch
    n = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        plan.align_t(a, tmpl, None, bands, st, 10)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(n):
        g.replay()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"eager {1e3 * (t1 - t0) / n:.3f} ms, graph {1e3 * (t2 - t1) / n:.3f} ms per call")
    plan.close()
