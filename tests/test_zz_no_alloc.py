"""guide_sample_noalloc (the entry point for callers that cannot allocate
device memory) through the C ABI: its outputs equal guide_sample's bit for
bit on two calls in a row, the second with a smaller queue (and another N),
so the shared scratch (counter, direction tables) carries nothing over."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_noalloc_matches_guide_sample():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_06997_amd as w
    dev = torch.device("cuda:0")
    room = synth.room(n_boxes=16)
    g = w.svo_build(room, 8)
    sp = [torch.from_numpy(a).to(dev) for a in synth.room_splats(room, 200_000, 5)]
    w.svo_accumulate(g, *sp)
    pos = torch.from_numpy(synth.area_points(room, 20000, 9)[0]).to(dev)
    for n, N, seed, bounce in [(20000, 16, 7, 0), (3001, 8, 8, 1), (777, 32, 8, 2), (65, 16, 9, 3)]:
        q = pos[:, :n].contiguous()
        d0, p0 = w.guide_sample(g, q, w.make_opts(N=N), seed=seed, bounce=bounce)
        d1 = torch.full((3, n), 7.0, device=dev)
        p1 = torch.full((n,), 7.0, device=dev)
        w.guide_sample_noalloc(g, q, w.make_opts(N=N), seed, bounce, d1, p1)
        torch.cuda.synchronize()
        assert torch.equal(d0, d1) and torch.equal(p0, p1), (n, N)
    # options the kernels take in place of the table: jitter and blur
    q = pos[:, :1000].contiguous()
    o = w.make_opts(N=16, jitter_key=5, blur=True)
    d0, p0 = w.guide_sample(g, q, o, seed=3, bounce=4)
    d1, p1 = torch.empty_like(d0), torch.empty_like(p0)
    w.guide_sample_noalloc(g, q, o, 3, 4, d1, p1)
    assert torch.equal(d0, d1) and torch.equal(p0, p1)
    # n = 0 is a no-op; mode 1 and N beyond the tables are rejected
    e = torch.empty((3, 0), device=dev)
    w.guide_sample_noalloc(g, e, w.make_opts(N=16), 1, 0, torch.empty((3, 0), device=dev),
                           torch.empty((0,), device=dev))
    with pytest.raises(w.WfpgError) as ei:
        w.guide_sample_noalloc(g, q, w.make_opts(N=16, mode=1), 1, 0, d1, p1)
    assert ei.value.status == -5
    with pytest.raises(w.WfpgError) as ei:
        w.guide_sample_noalloc(g, q, w.make_opts(N=64), 1, 0, d1, p1)
    assert ei.value.status == -1
    assert g.stats()["errors"] == 0
