"""GPU parity of positional binning (Alg. 2) and per-bin guiding (Alg. 3),
through the C ABI, against the oracle.

Bars: bins (node) and origins bit-exact; each member's pdf within 1e-5
relative of the oracle's (FP32 field of the same origin); sampled bins equal
except inside the FP32 scan band at CDF boundaries; directions within 2e-6
rad of the oracle's FP64 decode.
"""
import numpy as np
import pytest

import bars
import synth

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def w():
    import paper_2405_06997_amd as w
    w.lib()
    return w


def dev(torch_dev, a):
    torch, d = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a)).to(d)


@pytest.fixture(scope="module")
def c1(orc, w, torch_dev):
    rects = synth.cornell_box()
    D = 6
    o = orc.SVO(rects, D)
    xyz, em = o.leaf_info()
    sp = synth.leaf_splats(xyz, o.normals(D), em, D, seed=2)
    assert o.accumulate(*sp) == 0
    o.propagate()
    g = w.svo_build(rects, D)
    w.svo_accumulate(g, *[dev(torch_dev, a) for a in sp])
    pos, _, _ = synth.area_points(rects, 4096, 3)
    extra = np.random.default_rng(8).uniform(0.3, 0.7, (3, 37)).astype(np.float32)   # ragged, off-surface
    pos = np.ascontiguousarray(np.concatenate([pos, extra], 1))
    return dict(o=o, g=g, pos=pos, D=D)


def to_level_index(g, bins):
    sizes = np.array(g.level_sizes(), np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)])
    lv = np.searchsorted(off, bins, side="right") - 1
    return lv.astype(np.int32), (bins - off[lv]).astype(np.int64)


@pytest.mark.parametrize("c_ray,l_min", [(1, 0), (16, 2), (128, 3), (600, 1), (10 ** 6, 4), (40, 6)])
def test_partition_bitexact(c1, w, torch_dev, c_ray, l_min):
    o, g, pos = c1["o"], c1["g"], c1["pos"]
    b, org = w.partition(g, dev(torch_dev, pos), c_ray, l_min, seed=9, bounce=3)
    lv, ix = to_level_index(g, b.cpu().numpy().astype(np.int64))
    olv, oix = o.partition(pos, c_ray, l_min)
    assert np.array_equal(lv, olv) and np.array_equal(ix, oix)
    r = o.binned_sample(pos, c_ray, l_min, 8, 9, 3)
    assert np.array_equal(org.cpu().numpy().astype(np.int64), r["origin"])


@pytest.mark.parametrize("N,c_ray,l_min", [(8, 64, 3), (16, 64, 3), (32, 256, 2), (64, 256, 2), (128, 1024, 1)])
def test_binned_sample_matches_oracle(c1, w, torch_dev, N, c_ray, l_min):
    o, g, pos = c1["o"], c1["g"], c1["pos"]
    seed, bounce = 21, 2
    d, p, b = w.guide_sample_binned(g, dev(torch_dev, pos), w.bin_opts(N=N, c_ray=c_ray, l_min=l_min), seed,
                                    bounce, bins=True)
    d, p = d.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64)
    r = o.binned_sample(pos, c_ray, l_min, N, seed, bounce)
    lv, ix = to_level_index(g, b.cpu().numpy().astype(np.int64))
    assert np.array_equal(lv, r["level"]) and np.array_equal(ix, r["index"])
    # the sampled bin of each member: oracle bin unless inside the scan band
    import oracle
    uv = oracle.oct_encode_many(d)
    gb = np.minimum((uv * N).astype(np.int64), N - 1)
    same = (gb[0] == r["bin"][:, 0]) & (gb[1] == r["bin"][:, 1])
    band = (r["margin"] < bars.scan_band_seq(N)).any(1)
    assert (same | band).all(), np.nonzero(~(same | band))[0][:10]
    assert same.mean() > 0.999
    rel = np.abs(p[same] - r["pdf"][same]) / r["pdf"][same]
    bars.record(f"binned N={N} rel", rel.max())
    assert rel.max() <= bars.PDF_RTOL
    chord = np.linalg.norm(d[:, same] - r["dir"][:, same], axis=0)   # FP32 vectors are not unit exactly
    bars.record(f"binned N={N} dir", chord.max(), bars.DIR_TOL)
    assert chord.max() < bars.DIR_TOL, chord.max()


def test_binned_full_size_queue(orc, w, torch_dev):
    """The frame-scale room and camera queue with the paper's c_ray = 512 and
    l_min = 5: bins bit-exact against the oracle for every vertex; fields
    checked on sampled bins."""
    room = synth.room()
    o = orc.SVO(room, 10)
    sp = synth.room_splats(room, 2_000_000, 13)
    o.accumulate(*sp)
    o.propagate()
    g = w.svo_build(room, 10)
    w.svo_accumulate(g, *[dev(torch_dev, a) for a in sp])
    cam, _, _ = synth.camera_queue(room)
    dpos = dev(torch_dev, cam)
    b, org = w.partition(g, dpos, 512, 5, seed=4, bounce=0)
    lv, ix = to_level_index(g, b.cpu().numpy().astype(np.int64))
    olv, oix = o.partition(cam, 512, 5)
    assert np.array_equal(lv, olv) and np.array_equal(ix, oix)
    nb = len(np.unique(b.cpu().numpy()))
    assert 100 < nb < cam.shape[1] // 64
    d, p, bb = w.guide_sample_binned(g, dpos, w.bin_opts(N=16, c_ray=512, l_min=5), 4, 0, bins=True)
    assert (p > 0).all() and np.array_equal(bb.cpu().numpy(), b.cpu().numpy())
    # a strided sample of members: pdf = the oracle field of its origin at the sampled bin
    i = np.arange(0, cam.shape[1], cam.shape[1] // 256)
    orig = org.cpu().numpy()[i]
    f = o.guide_pdf(cam[:, orig], 16)
    import oracle
    uv = oracle.oct_encode_many(d.cpu().numpy().astype(np.float64)[:, i])
    gb = np.minimum((uv * 16).astype(np.int64), 15)
    frac = uv * 16 - np.floor(uv * 16)
    eb = bars.edge_band(16)
    inner = ((frac > eb) & (frac < 1 - eb)).all(0)
    want = f[np.arange(len(i)), gb[1] * 16 + gb[0]]
    np.testing.assert_allclose(p.cpu().numpy()[i][inner], want[inner], rtol=bars.PDF_RTOL)


def test_binned_errors(c1, w, torch_dev):
    g, pos = c1["g"], dev(torch_dev, c1["pos"])
    for bad in (dict(N=12), dict(c_ray=0), dict(l_min=7), dict(eps=0.0)):
        kw = dict(N=16, c_ray=64, l_min=3)
        kw.update(bad)
        with pytest.raises(w.WfpgError):
            w.guide_sample_binned(g, pos, w.bin_opts(**kw), 0, 0)
    d, p = w.guide_sample_binned(g, pos[:, :0].contiguous(), w.bin_opts(), 0, 0)
    assert d.shape == (3, 0)
