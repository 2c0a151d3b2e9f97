"""Uneven batches (bh_align_uneven through UnevenAligner): particles of three
box sizes and bandlimits marched together, one launch per band.

Bar: bit-for-bit the result of aligning each box size separately with its
own plan over the bands up to its bandlimit (both in the batch-invariant
forms, so the wave split does not depend on how many particles share a
launch).  Also the error paths of the ordering rules.
"""

import numpy as np
import pytest

import synth
from gpu_util import cuda_device, say

pytestmark = pytest.mark.gpu

BOXES = {16: 6, 20: 8, 24: 10}
P, STEPS = 24, 8


def _data(dev):
    import torch
    rng = np.random.default_rng(17)
    blobs = [synth.blob_template(rng, 10), synth.blob_template(rng, 14)]
    groups = {}
    for j, N in enumerate(BOXES):
        n = 5 + 2 * j
        g = synth.quat_to_matrix(synth.haar_quaternions(rng, n))
        t = rng.integers(0, 2, n)
        vols = np.stack([synth.add_noise(synth.render_blobs(blobs[t[i]], N, g[i]), 0.5, rng)
                         for i in range(n)]).astype(np.float32)
        st = synth.matrix_to_euler_zyz(synth.quat_to_matrix(synth.haar_quaternions(rng, n * P)))
        groups[N] = (torch.from_numpy(vols).to(dev), t.astype(np.int32),
                     torch.from_numpy(st.reshape(n, P, 3)).to(dev))
    tv = {N: np.stack([synth.render_blobs(b, N) for b in blobs]).astype(np.float32) for N in BOXES}
    return groups, tv


def test_uneven_equals_separate_boxes():
    import torch
    from paper_2509_01180_amd.api import Plan
    from paper_2509_01180_amd.uneven import Group, UnevenAligner
    dev = cuda_device()
    groups, tv = _data(dev)
    plans = {N: Plan(N, L, device=0) for N, L in BOXES.items()}
    tmpl = {N: plans[N].expand(torch.from_numpy(tv[N]).to(dev), ) for N in BOXES}
    say(f"uneven align over boxes {sorted(BOXES)} (L {sorted(BOXES.values())})")
    ua = UnevenAligner(plans, tmpl, step=3)
    assert ua.bands == [3, 6, 8, 9, 10]
    order = [20, 16, 24]            # groups in any order
    res = ua.align([Group(N, groups[N][0], groups[N][1], groups[N][2]) for N in order], STEPS,
                   batch_invariant=True)
    torch.cuda.synchronize()
    for (N, (eu, sc)) in zip(order, res):
        vols, t, st = groups[N]
        plan = plans[N]
        a = plan.expand_ex(vols, "fp32", batch_invariant=True)
        bands = [b for b in ua.bands if b <= BOXES[N]]
        e_ref, s_ref = plan.align_t(a, tmpl[N], torch.from_numpy(t).to(dev), bands, st, STEPS,
                                    batch_invariant=True)
        torch.cuda.synchronize()
        assert torch.equal(eu, e_ref), N
        assert torch.equal(sc, s_ref), N
    for p in plans.values():
        p.close()


def test_uneven_ordering_errors():
    import torch
    from paper_2509_01180_amd.api import Plan
    from paper_2509_01180_amd._lib import BhError
    dev = cuda_device()
    plan = Plan(16, 8, device=0)
    a = torch.zeros((3, plan.C, 2), dtype=torch.float32, device=dev)
    t = torch.zeros((1, plan.C, 2), dtype=torch.float32, device=dev)
    st = torch.zeros((3, 4, 3), dtype=torch.float64, device=dev)
    with pytest.raises(BhError):       # increasing bandlimits
        plan.align_uneven(a, [4, 8, 8], t, None, [4, 8], st, 2)
    with pytest.raises(BhError):       # a particle below the first band
        plan.align_uneven(a, [8, 8, 3], t, None, [4, 8], st, 2)
    with pytest.raises(BhError):       # bands not increasing
        plan.align_uneven(a, [8, 8, 8], t, None, [8, 4], st, 2)
    eu, sc = plan.align_uneven(a, [8, 6, 4], t, None, [4, 6, 8], st, 2)
    torch.cuda.synchronize()
    assert torch.all(torch.isfinite(eu))
    plan.close()


def test_uneven_graph_replays_match_eager():
    """The uneven march captured once (GraphedAlignUneven) and replayed on
    refilled inputs gives the eager call's bits on every replay."""
    import torch
    from paper_2509_01180_amd.api import Plan
    from paper_2509_01180_amd.graphs import GraphedAlignUneven
    from paper_2509_01180_amd.uneven import Group, UnevenAligner
    dev = cuda_device()
    groups, tv = _data(dev)
    plans = {N: Plan(N, L, device=0) for N, L in BOXES.items()}
    tmpl = {N: plans[N].expand(torch.from_numpy(tv[N]).to(dev)) for N in BOXES}
    ua = UnevenAligner(plans, tmpl, step=3)
    say(f"uneven graph capture over boxes {sorted(BOXES)}")
    sets = []
    for flip in (False, True):
        gs = []
        for N in BOXES:
            vols, t, st = groups[N]
            gs.append(Group(N, torch.flip(vols, dims=(1,)).contiguous() if flip else vols, t,
                            st.flip(1).contiguous() if flip else st))
        sets.append(ua.pack(gs, batch_invariant=True))
    a, Lp, ti, bands, st, _rows = sets[0]
    a_buf, st_buf = a.clone(), st.clone()
    g = GraphedAlignUneven(ua.top, a_buf, Lp, ua.table, ti, bands, st_buf, STEPS,
                           batch_invariant=True)
    ref = [ua.top.align_uneven(x[0], x[1], ua.table, x[2], x[3], x[4], STEPS, batch_invariant=True)
           for x in sets]
    torch.cuda.synchronize()
    for rep in range(4):
        k = rep % 2
        a_buf.copy_(sets[k][0])
        st_buf.copy_(sets[k][4])
        eu, sc = g.replay()
        torch.cuda.synchronize()
        assert torch.equal(eu, ref[k][0]) and torch.equal(sc, ref[k][1]), rep
    for p in plans.values():
        p.close()
