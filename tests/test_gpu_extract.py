"""GPU parity of exitance extraction (Eq. 5, svo_accumulate_paths) through the
C ABI: the leaf accumulators after a wavefront's path memory is splatted
equal the oracle's accumulation of the oracle's Eq. 5 splats (counts and
dropped bit-exact, FP32 sums within the atomic-order bound (count-1) * u *
sum), and the propagated exitance of every level within 1e-5.
"""
import numpy as np
import pytest

import oracle
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


def compare(o, g, D):
    s, cnt = g.export_accum()
    _, s64, ocnt = o.leaf_accum()
    assert np.array_equal(cnt.astype(np.int64), ocnt)
    assert g.stats()["dropped"] == o.dropped()
    bound = np.maximum(ocnt - 1, 0) * 2.0 ** -24 * s64 + 1e-30
    assert (np.abs(s.astype(np.float64) - s64) <= bound * 1.0001).all()
    for l in range(D + 1):
        _, _, ex = g.export_level(l)
        e32, _ = o.exitance(l)
        assert (np.abs(ex - e32) / np.maximum(np.abs(e32), 1e-30)).max() < 1e-5, l


@pytest.mark.parametrize("scene,D,P,d", [("box", 6, 20000, 8), ("box", 5, 3001, 3), ("room", 10, 400000, 8)])
def test_accumulate_paths_matches_oracle(orc, w, torch_dev, scene, D, P, d):
    rects = synth.cornell_box() if scene == "box" else synth.room()
    pos, T, eye, hit, Le = synth.path_wavefront(rects, P, d, seed=P)
    # a few invalid vertices: outside the cube, non-finite throughput
    pos[0, 0, :5] = 1.5
    T[1, 2, 5:9] = np.inf
    o = orc.SVO(rects, D)
    o.accumulate(*oracle.path_splats(pos, T, eye, hit, Le))
    o.propagate()
    g = w.svo_build(rects, D)
    w.svo_accumulate_paths(g, *[dev(torch_dev, a) for a in (pos, T, eye, hit, Le)])
    compare(o, g, D)
    assert o.dropped() > 0


def test_accumulate_paths_equals_splatting_the_eq5_splats(orc, w, torch_dev):
    rects = synth.cornell_box()
    pos, T, eye, hit, Le = synth.path_wavefront(rects, 5000, 6, seed=3)
    g1 = w.svo_build(rects, 6)
    w.svo_accumulate_paths(g1, *[dev(torch_dev, a) for a in (pos, T, eye, hit, Le)])
    g2 = w.svo_build(rects, 6)
    w.svo_accumulate(g2, *[dev(torch_dev, a) for a in oracle.path_splats(pos, T, eye, hit, Le)])
    s1, c1 = g1.export_accum()
    s2, c2 = g2.export_accum()
    assert np.array_equal(c1, c2)
    np.testing.assert_allclose(s1, s2, rtol=1e-5)


def test_accumulate_paths_edges(w, torch_dev):
    rects = synth.cornell_box()
    g = w.svo_build(rects, 5)
    pos, T, eye, hit, Le = synth.path_wavefront(rects, 100, 4, seed=1)
    none = np.full(100, -1, np.int32)
    w.svo_accumulate_paths(g, *[dev(torch_dev, a) for a in (pos, T, eye, none, Le)])
    _, cnt = g.export_accum()
    assert cnt.sum() == 0 and g.stats()["dropped"] == 0
    assert w.lib().svo_accumulate_paths(g.handle, None, None, None, None, None, 10, 4, None) == -1
    assert w.lib().svo_accumulate_paths(g.handle, None, None, None, None, None, 0, 0, None) == -1
    empty = w.svo_build(rects[:0], 5)     # no leaves: every splat is dropped
    w.svo_accumulate_paths(empty, *[dev(torch_dev, a) for a in (pos, T, eye, hit, Le)])
    assert empty.stats()["dropped"] == int(hit[hit >= 1].sum())
