"""Batched bounces in a captured HIP graph, and the launch-shape autotuner.

The graph's kernels read their queue lengths from device memory; every
replay (with eager work and synchronizations in between) must equal eager
guide_sample bit for bit, also after the lengths shrink, and every bounce of
the eight-bounce wavefront on the depth-10 room must match the oracle."""
import numpy as np
import pytest

import bars
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_06997_amd as w
    dev = torch.device("cuda:0")
    room = synth.room(n_boxes=16)
    g = w.svo_build(room, 8)
    sp = [torch.from_numpy(a).to(dev) for a in synth.room_splats(room, 200_000, 5)]
    w.svo_accumulate(g, *sp)
    return torch, dev, w, room, g, sp


def test_graph_replays_match_eager(env):
    torch, dev, w, room, g, sp = env
    sizes = [5000, 3001, 777, 64, 1]
    Ns = [16, 8, 32, 16, 8]
    queues = [torch.from_numpy(synth.area_points(room, n, 40 + b)[0]).to(dev)
              for b, n in enumerate(sizes)]
    n_dev = torch.tensor(sizes, dtype=torch.int64, device=dev)
    G = w.BounceGraph(g, queues, n_dev, Ns, seed=99)

    def eager(b, n):
        return w.guide_sample(g, queues[b][:, :n].contiguous(), w.make_opts(N=Ns[b]), seed=99, bounce=b)

    for rep in range(3):
        G.launch()
        torch.cuda.synchronize()
        for b, n in enumerate(sizes):
            d, p = eager(b, n)
            assert torch.equal(G.dirs[b][:, :n], d), (rep, b)
            assert torch.equal(G.pdfs[b][:n], p), (rep, b)
        w.svo_accumulate(g, sp[0][:, :0].contiguous(), sp[1][:, :0].contiguous(),
                         sp[2][:, :0].contiguous())   # eager work between replays
        torch.cuda.synchronize()
    # shrink the queues on the device: the same graph handles the new lengths
    new = [1234, 0, 500, 64, 1]
    n_dev.copy_(torch.tensor(new, dtype=torch.int64))
    G.dirs[0].fill_(7.0)
    G.launch()
    torch.cuda.synchronize()
    for b, n in enumerate(new):
        if n == 0:
            continue
        d, p = eager(b, n)
        assert torch.equal(G.dirs[b][:, :n], d) and torch.equal(G.pdfs[b][:n], p)
    assert (G.dirs[0][:, new[0]:] == 7.0).all()   # nothing written past the live length
    assert g.stats()["errors"] == 0
    G.close()


def test_autotune_and_tiles(env):
    torch, dev, w, room, g, sp = env
    pos = torch.from_numpy(synth.area_points(room, 20000, 3)[0]).to(dev)
    ref_d, ref_p = w.guide_sample(g, pos, w.make_opts(N=16), seed=1, bounce=0)
    pos2k = pos[:, :2000].contiguous()
    pos4k = pos[:, :4000].contiguous()
    ref_pdf = w.guide_pdf(g, pos2k, w.make_opts(N=16))
    ref_other = {N: w.guide_sample(g, pos4k, w.make_opts(N=N), seed=1, bounce=0) for N in (8, 32)}
    best = w.autotune(g, pos, 16, reps=1)
    assert best["ms"] > 0
    assert w.get_tile(g, 16)["waves_per_block"] == best["waves_per_block"]
    # results do not depend on the launch shape (odd wave counts too: the
    # per-wave LDS arrays stay aligned whatever the slot count)
    for tile in [(1, 2), (6, 16), (4, 8), (2, 4), (16, 2), (3, 8), (5, 4), (7, 3)]:
        w.set_tile(g, 16, *tile)
        d, p = w.guide_sample(g, pos, w.make_opts(N=16), seed=1, bounce=0)
        assert torch.equal(d, ref_d) and torch.equal(p, ref_p)
        pp = w.guide_pdf(g, pos2k, w.make_opts(N=16))
        assert torch.equal(pp, ref_pdf)
    for tile in [(3, 8), (5, 4)]:   # N = 8 (eight slots) and N = 32 (two)
        for N in (8, 32):
            w.set_tile(g, N, *tile)
            d, p = w.guide_sample(g, pos4k, w.make_opts(N=N), seed=1, bounce=0)
            assert torch.equal(d, ref_other[N][0]) and torch.equal(p, ref_other[N][1])
    for bad in [(0, 2), (17, 2), (4, 0), (4, 65)]:
        with pytest.raises(w.WfpgError):
            w.set_tile(g, 16, *bad)


def test_autotune_picks_finest_N_within_budget(env):
    torch, dev, w, room, g, sp = env
    q = torch.from_numpy(synth.area_points(room, 20000, 61)[0]).to(dev)
    r = w.autotune_n(g, q, 1e9)
    assert r["N"] == 32
    ms = r["ms_per_N"]
    assert ms[8] < ms[32]        # 16x the bins
    assert w.autotune_n(g, q, 0.0)["N"] == 8
    mid = (ms[16] * 1e6 / 20000) * 1.000001
    pick = w.autotune_n(g, q, mid)["N"]   # re-timed: 16 unless timing noise moves a neighbour
    assert pick in (8, 16, 32)
    t = w.get_tile(g, r["N"])
    assert t["waves_per_block"] >= 1


def test_autotune_n_on_a_large_queue_uses_a_subset(env):
    """Above 2 x 262,144 vertices the tile sweep runs on a strided subset; the
    whole queue is then timed per N."""
    torch, dev, w, room, g, sp = env
    q = torch.from_numpy(synth.area_points(room, 600_000, 62)[0]).to(dev)
    ref_d, ref_p = w.guide_sample(g, q, w.make_opts(N=8), seed=2, bounce=1)
    r = w.autotune_n(g, q, 1e9, reps=1)
    assert r["N"] == 32 and all(v > 0 for v in r["ms_per_N"].values())
    d, p = w.guide_sample(g, q, w.make_opts(N=8), seed=2, bounce=1)
    assert torch.equal(d, ref_d) and torch.equal(p, ref_p)


def test_graph_eight_bounces_match_oracle(orc):
    """The batching configuration: the depth-10 room with 2M splats, bounce 0
    the 1920 x 1080 camera queue, bounces 1-7 area-uniform queues shrinking
    by U[0.5, 0.8] per bounce, N per bounce in {8, 16, 32}, replayed twice
    from one captured graph. On every bounce a strided subset (at least 4096
    vertices; the oracle's counter is the queue index and its bounce the
    bounce number) matches the oracle at the sampling bars."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_2405_06997_amd as w
    dev = torch.device("cuda:0")
    room = synth.room()
    o = orc.SVO(room, 10)
    sp = synth.room_splats(room, 2_000_000, 13)
    o.accumulate(*sp)
    o.propagate()
    _, _, cnt = o.leaf_accum()
    C = int(max(1, cnt.max()))
    g = w.svo_build(room, 10)
    w.svo_accumulate(g, *[torch.from_numpy(a).to(dev) for a in sp])
    cam, cnrm, _ = synth.camera_queue(room)
    qs, sizes = synth.bounce_queues(room, cam, cnrm, 8, 15)
    Ns = [16, 8, 32, 16, 8, 32, 16, 8]
    queues = [torch.from_numpy(np.ascontiguousarray(p)).to(dev) for p, _ in qs]
    n_dev = torch.tensor(sizes, dtype=torch.int64, device=dev)
    G = w.BounceGraph(g, queues, n_dev, Ns, seed=4242)
    for rep in range(2):
        G.launch()
        torch.cuda.synchronize()
        for b, (n, N) in enumerate(zip(sizes, Ns)):
            step = max(1, n // 4096)
            idx = np.arange(0, n, step)
            if len(idx) < 4096:
                idx = np.arange(n)
            pos = np.ascontiguousarray(qs[b][0][:, idx])
            ref = o.guide_sample(pos, N, seed=4242, bounce=b, counter=idx)
            d = G.dirs[b][:, idx].cpu().numpy().astype(np.float64)
            p = G.pdfs[b][idx].cpu().numpy().astype(np.float64)
            uv = oracle.oct_encode_many(d)
            gb = np.minimum((uv * N).astype(np.int64), N - 1)
            same = (gb[0] == ref["bin"][:, 0]) & (gb[1] == ref["bin"][:, 1])
            band = ref["margin"].min(1) < bars.scan_band(N, C)
            fx, fy = uv[0] * N, uv[1] * N
            edge = np.minimum(np.abs(fx - np.rint(fx)), np.abs(fy - np.rint(fy)))
            bad = ~same & ~band & (edge > bars.edge_band(N))
            assert not bad.any(), (rep, b, np.nonzero(bad)[0][:10])
            assert same.mean() > 0.99, (rep, b)
            rel = np.abs(p[same] - ref["pdf"][same]) / ref["pdf"][same]
            bars.record(f"bounce graph N={N} rel", rel.max(), bars.pdf_bound(N, C))
            assert rel.max() <= bars.PDF_RTOL, (rep, b, rel.max())
            ok = same & (edge > bars.edge_band(N))
            chord = np.linalg.norm(d[:, ok] - ref["dir"][:, ok], axis=0)
            bars.record(f"bounce graph N={N} dir", chord.max(), bars.DIR_TOL)
            assert chord.max() < bars.DIR_TOL, (rep, b, chord.max())
    assert g.stats()["errors"] == 0
    G.close()


def test_binned_depth_halving_graph(orc):
    """Alg. 1 with Alg. 2 and 3 per bounce: binned guiding with the field
    resolution halved per depth (128, 64, 32, 16; c_ray = 256, l_min = 3)
    over shrinking queues, captured once in a HIP graph and replayed (eager
    work and synchronizations between replays). Every replay equals the eager
    calls bit for bit, and every member's bin, pdf and direction match the
    oracle's binned sampler (sequential-scan band, 2e-6 directions)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_2405_06997_amd as w
    dev = torch.device("cuda:0")
    room = synth.room(n_boxes=16)
    D = 8
    o = orc.SVO(room, D)
    xyz, em = o.leaf_info()
    sp = synth.leaf_splats(xyz, o.normals(D), em, D, seed=2)
    assert o.accumulate(*sp) == 0
    o.propagate()
    g = w.svo_build(room, D)
    w.svo_accumulate(g, *[torch.from_numpy(a).to(dev) for a in sp])
    Ns = [128, 64, 32, 16]
    sizes = [24000, 15000, 9000, 5000]
    qs = [synth.area_points(room, n, 70 + b)[0] for b, n in enumerate(sizes)]
    pos = [torch.from_numpy(q).to(dev) for q in qs]
    opts = [w.bin_opts(N=N, c_ray=256, l_min=3) for N in Ns]
    dirs = [torch.empty((3, n), device=dev) for n in sizes]
    pdfs = [torch.empty((n,), device=dev) for n in sizes]

    def frame():
        for b in range(4):
            w.guide_sample_binned(g, pos[b], opts[b], seed=808, bounce=b, dir_out=dirs[b], pdf_out=pdfs[b])

    frame()   # eager: grows the binning scratch to these sizes before capture
    torch.cuda.synchronize()
    eager = [(d.clone(), p.clone()) for d, p in zip(dirs, pdfs)]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        frame()
    for rep in range(3):
        for d, p in zip(dirs, pdfs):
            d.fill_(7.0)
            p.fill_(7.0)
        graph.replay()
        torch.cuda.synchronize()
        for b in range(4):
            assert torch.equal(dirs[b], eager[b][0]) and torch.equal(pdfs[b], eager[b][1]), (rep, b)
        w.guide_sample(g, pos[3][:, :100].contiguous(), w.make_opts(N=8), seed=1, bounce=0)   # eager work
        torch.cuda.synchronize()
    for b, N in enumerate(Ns):
        r = o.binned_sample(qs[b], 256, 3, N, 808, b)
        d = dirs[b].cpu().numpy().astype(np.float64)
        p = pdfs[b].cpu().numpy().astype(np.float64)
        uv = oracle.oct_encode_many(d)
        gb = np.minimum((uv * N).astype(np.int64), N - 1)
        same = (gb[0] == r["bin"][:, 0]) & (gb[1] == r["bin"][:, 1])
        band = (r["margin"] < bars.scan_band_seq(N)).any(1)
        assert (same | band).all(), (N, np.nonzero(~(same | band))[0][:10])
        assert same.mean() > 0.999
        rel = np.abs(p[same] - r["pdf"][same]) / r["pdf"][same]
        bars.record(f"binned graph N={N} rel", rel.max())
        assert rel.max() <= bars.PDF_RTOL
        chord = np.linalg.norm(d[:, same] - r["dir"][:, same], axis=0)
        assert chord.max() < bars.DIR_TOL, chord.max()
    assert g.stats()["errors"] == 0
