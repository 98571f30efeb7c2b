"""GPU-vs-oracle parity of the HIP path, called through the C ABI.

Bars (derived in tests/bars.py): SVO build arrays, traversal records and bin
choices bit-exact; PDFs within 1e-5 relative (FP32 field, FP32 CDF; the
arithmetic's worst case, recorded beside the measured maximum, is far
inside it); sampled bins equal except where the oracle's target lies inside
the FP32 scan band of a CDF boundary (several answers are then correct);
sampled directions within 2e-6 rad of the oracle's FP64 decode; pdf_eval's
bin equal except within 8 ulps of x N of a bin edge.
"""
import math

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


def to_dev(torch_dev, *arrs):
    torch, dev = torch_dev
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrs]


@pytest.fixture(scope="module")
def c1(orc, w, torch_dev):
    """Tiny Cornell box, depth 6, one splat per (leaf, side)."""
    box = synth.cornell_box()
    o = orc.SVO(box, 6)
    xyz, em = o.leaf_info()
    sp = synth.leaf_splats(xyz, o.normals(6), em, 6, seed=2)
    assert o.accumulate(*sp) == 0
    o.propagate()
    g = w.svo_build(box, 6)
    w.svo_accumulate(g, *to_dev(torch_dev, *sp))
    pos, nrm, _ = synth.area_points(box, 4096, 3)
    return dict(rects=box, o=o, g=g, pos=pos, nrm=nrm, D=6, splats=sp)


@pytest.fixture(scope="module")
def c2(orc, w, torch_dev):
    """Room, depth 10 (~8M leaves), 2M splats."""
    room = synth.room()
    o = orc.SVO(room, 10)
    sp = synth.room_splats(room, 2_000_000, 13)
    dropped = o.accumulate(*sp)
    o.propagate()
    g = w.svo_build(room, 10)
    w.svo_accumulate(g, *to_dev(torch_dev, *sp))
    cam, cnrm, _ = synth.camera_queue(room)
    rnd, rnrm, _ = synth.area_points(room, 2_073_600, 14)
    _, _, cnt = o.leaf_accum()
    return dict(rects=room, o=o, g=g, D=10, cam=cam, rnd=rnd, dropped=dropped, splats=sp,
                C=int(max(1, cnt.max())))


def sample_cols(a, k, seed=0):
    idx = np.random.default_rng(seed).choice(a.shape[1], size=k, replace=False)
    idx.sort()
    return np.ascontiguousarray(a[:, idx]), idx


# ------------------------------------------------------------------ build ----
@pytest.mark.parametrize("case", ["c1", "c2"])
def test_build_bitexact(case, request):
    c = request.getfixturevalue(case)
    o, g, D = c["o"], c["g"], c["D"]
    assert g.level_sizes() == o.level_sizes()
    for l in range(D + 1):
        keys, nrm, _ = g.export_level(l)
        assert np.array_equal(keys, o.keys(l)), l
        assert np.array_equal(nrm.view(np.uint32), o.normals(l).view(np.uint32)), l
    st = g.stats()
    assert st["leaves"] == o.level_size(D) and st["errors"] == 0


def test_build_other_depths(orc, w):
    rng = np.random.default_rng(5)
    for D in (1, 3, 5, 8):
        rs = synth.room(n_boxes=8)
        o = orc.SVO(rs, D)
        g = w.svo_build(rs, D)
        assert g.level_sizes() == o.level_sizes()
        for l in range(D + 1):
            k, n, _ = g.export_level(l)
            assert np.array_equal(k, o.keys(l))
            assert np.array_equal(n.view(np.uint32), o.normals(l).view(np.uint32))


# ------------------------------------------------------------- accumulate ----
def test_accumulate_one_splat_per_side_bitexact(c1):
    o, g = c1["o"], c1["g"]
    s, cnt = g.export_accum()
    assert (cnt == 1).all()
    for l in range(7):
        _, _, ex = g.export_level(l)
        e32, _ = o.exitance(l)
        assert np.array_equal(ex.view(np.uint32), e32.view(np.uint32)), l


def test_accumulate_room_counts_and_sums(c2):
    o, g = c2["o"], c2["g"]
    s, cnt = g.export_accum()
    s32, s64, ocnt = o.leaf_accum()
    assert np.array_equal(cnt.astype(np.int64), ocnt)
    assert g.stats()["dropped"] == c2["dropped"] == o.dropped()
    # FP32 atomics: |sum - exact| <= (count - 1) * u * sum
    u = 2.0 ** -24
    bound = np.maximum(ocnt - 1, 0) * u * s64 + 1e-30
    assert (np.abs(s.astype(np.float64) - s64) <= bound * 1.0001).all()
    for l in range(11):
        _, _, ex = g.export_level(l)
        e32, _ = o.exitance(l)
        denom = np.maximum(np.abs(e32), 1e-30)
        assert (np.abs(ex - e32) / denom).max() < 1e-5, l


# ------------------------------------------------------------------ march ----
def _march_compare(o, g, w, torch_dev, pos, N):
    (dpos,) = to_dev(torch_dev, pos)
    rec, vis = w.debug_march(g, dpos, w.make_opts(N=N))
    rec = rec.cpu().numpy().astype(np.int64)
    vis = vis.cpu().numpy().astype(np.int64)
    want, wvis = o.debug_march(pos, N, lds_levels=5, hier=False, visits=True)
    hit = want[..., 0] == 1
    assert np.array_equal(rec[..., 0], want[..., 0])
    assert np.array_equal(rec[hit], want[hit])
    assert np.array_equal(vis, wvis)
    assert g.stats()["errors"] == 0
    return hit.mean()


def test_march_bitexact_c1(c1, w, torch_dev):
    for N in (8, 16):
        hr = _march_compare(c1["o"], c1["g"], w, torch_dev, c1["pos"], N)
        assert hr > 0.3


def test_march_bitexact_on_planes(c1, w, torch_dev):
    """Queries exactly on cell planes, where the march's mirrored frame must
    reproduce the original frame's half-open cells: the corners of the 1/4,
    1/8 and leaf (1/64) grids, the cube's faces, and random points with some
    coordinates snapped to leaf planes; every record and visit count bit-exact."""
    rng = np.random.default_rng(17)
    g4 = np.stack(np.meshgrid(*[np.arange(5) / 4] * 3, indexing="ij")).reshape(3, -1)
    g8 = np.stack(np.meshgrid(*[np.arange(9) / 8] * 3, indexing="ij")).reshape(3, -1)
    leaf = rng.integers(0, 65, (3, 400)) / 64.0
    mix = np.where(rng.random((3, 400)) < 0.5, rng.integers(0, 65, (3, 400)) / 64.0, rng.random((3, 400)))
    pos = np.ascontiguousarray(np.concatenate([g4, g8, leaf, mix], 1).astype(np.float32))
    for N in (8, 16):
        _march_compare(c1["o"], c1["g"], w, torch_dev, pos, N)


@pytest.mark.parametrize("N,k", [(16, 384), (8, 256), (32, 48)])
def test_march_bitexact_c2(c2, w, torch_dev, N, k):
    cam, _ = sample_cols(c2["cam"], k // 2, 1)
    rnd, _ = sample_cols(c2["rnd"], k // 2, 2)
    _march_compare(c2["o"], c2["g"], w, torch_dev, np.concatenate([cam, rnd], 1), N)


def test_march_counts_match_oracle(c2, w, torch_dev):
    """The per-vertex work counts used for the benchmark's algorithmic bytes
    equal the oracle's node-test and hit counts."""
    cam, _ = sample_cols(c2["cam"], 128, 21)
    (dpos,) = to_dev(torch_dev, cam)
    cnt = w.march_counts(c2["g"], dpos, w.make_opts(N=16)).cpu().numpy().astype(np.int64)
    rec, vis = c2["o"].debug_march(cam, 16, lds_levels=5, hier=False, visits=True)
    assert np.array_equal(cnt[:, 0], vis.sum(1))
    assert np.array_equal(cnt[:, 1], rec[..., 0].sum(1))


# -------------------------------------------------------------- guide_pdf ----
def _pdf_compare(o, g, w, torch_dev, pos, N, C=1, name="pdf", want=None):
    (dpos,) = to_dev(torch_dev, pos)
    got = w.guide_pdf(g, dpos, w.make_opts(N=N)).cpu().numpy().astype(np.float64)
    if want is None:
        want = o.guide_pdf(pos, N)
    rel = np.abs(got - want) / want
    bars.record(f"{name} N={N} rel", rel.max(), bars.pdf_bound(N, C))
    assert rel.max() <= bars.PDF_RTOL, rel.max()
    np.testing.assert_allclose(got.sum(1) * 4 * math.pi / N ** 2, 1.0, rtol=bars.PDF_RTOL)
    return rel.max()


def test_guide_pdf_c1(c1, w, torch_dev):
    for N in (8, 16, 32):
        _pdf_compare(c1["o"], c1["g"], w, torch_dev, c1["pos"][:, :1024], N, name="guide_pdf C1")


def test_guide_pdf_off_surface_and_on_planes(orc, c1, w, torch_dev):
    """Vertices the first step of the guide kernel treats apart: points in
    empty space (an empty origin leaf: every bin marched in full), points on
    leaf corners (on the planes of every level, crossings at t = 0 into a
    face neighbour) and points on the cube's faces (first crossing out of the
    cube), against the oracle's guide_pdf."""
    rng = np.random.default_rng(31)
    D = 6
    free = rng.random((3, 192))
    corner = np.round(rng.random((3, 192)) * 2 ** D) / 2 ** D
    face = rng.random((3, 96))
    face[rng.integers(0, 3, 96), np.arange(96)] = rng.integers(0, 2, 96)
    pos = np.ascontiguousarray(np.concatenate([free, corner, face], 1).astype(np.float32))
    for N in (8, 16):
        _pdf_compare(c1["o"], c1["g"], w, torch_dev, pos, N, name="guide_pdf off-surface C1")
    _sample_compare(orc, c1["o"], c1["g"], w, torch_dev, pos, 16, seed=77, bounce=3,
                    name="guide_sample off-surface C1")


@pytest.mark.parametrize("D", [1, 2, 3, 4, 8])
def test_guide_shallow_and_other_depths(orc, w, torch_dev, D):
    """guide_pdf and guide_sample on SVOs of other depths than the two
    configurations (depth 1 has no level-2 bitmap word; the first steps and
    the three-level window work on shallow trees too) against the oracle,
    for surface vertices and points anywhere in the cube."""
    rs = synth.room(n_boxes=8)
    o = orc.SVO(rs, D)
    xyz, em = o.leaf_info()
    sp = synth.leaf_splats(xyz, o.normals(D), em, D, seed=40 + D)
    assert o.accumulate(*sp) == 0
    o.propagate()
    g = w.svo_build(rs, D)
    w.svo_accumulate(g, *to_dev(torch_dev, *sp))
    area, _, _ = synth.area_points(rs, 256, 50 + D)
    free = np.random.default_rng(60 + D).random((3, 128))
    pos = np.ascontiguousarray(np.concatenate([area, free], 1).astype(np.float32))
    for N in (8, 16):
        _pdf_compare(o, g, w, torch_dev, pos, N, name=f"guide_pdf D={D}")
    _sample_compare(orc, o, g, w, torch_dev, pos, 16, seed=70 + D, bounce=1, name=f"guide_sample D={D}")


def test_guide_large_svo_four_byte_records(orc, w, torch_dev):
    """A room with 400 boxes at depth 10: 22 M nodes, more than 3-byte hit
    records can index, so N = 16 keeps 4-byte records (and five vertex
    slots); guide_pdf and guide_sample against the oracle, and the modes whose
    finalization builds the field in the slot's record memory: guide_pdf
    with the blur and the product sampler."""
    rs = synth.room(n_boxes=400)
    o = orc.SVO(rs, 10)
    assert sum(o.level_sizes()) >= 0xffffff
    sp = synth.room_splats(rs, 1_000_000, 17)
    o.accumulate(*sp)
    o.propagate()
    g = w.svo_build(rs, 10)
    w.svo_accumulate(g, *to_dev(torch_dev, *sp))
    assert g.stats()["nodes"] == sum(o.level_sizes())
    _, _, cnt = o.leaf_accum()
    C = int(max(1, cnt.max()))
    pos, _, _ = synth.area_points(rs, 192, 18)
    _pdf_compare(o, g, w, torch_dev, pos, 16, C, name="guide_pdf 22M-node room")
    _sample_compare(orc, o, g, w, torch_dev, pos, 16, seed=19, bounce=0, C=C, name="guide_sample 22M-node room")
    (dpos,) = to_dev(torch_dev, pos)
    got = w.guide_pdf(g, dpos, w.make_opts(N=16, blur=True)).cpu().numpy().astype(np.float64)
    L = o.field_aa(pos, 16, blur=True)
    want = L / L.sum(1, keepdims=True) * 256 / (4 * math.pi)
    rel = np.abs(got - want) / want
    bars.record("guide_pdf blur 22M-node room N=16 rel", rel.max(), bars.pdf_bound(16, C))
    assert rel.max() <= bars.PDF_RTOL, rel.max()
    nrm = np.random.default_rng(20).normal(size=pos.shape)
    nrm = (nrm / np.linalg.norm(nrm, axis=0)).astype(np.float32)
    (dnrm,) = to_dev(torch_dev, nrm)
    d, p = w.guide_sample_product(g, dpos, w.make_opts(N=16), 21, 1, nrm=dnrm)
    r = o.product_sample(pos, 16, 21, 1, nrm=nrm)
    d, p = d.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64)
    gb = np.minimum((orc.oct_encode_many(d) * 16).astype(np.int64), 15)
    same = (gb[0] == r["bin"][:, 0]) & (gb[1] == r["bin"][:, 1])
    band = (r["margin"] < bars.scan_band_seq(16)).any(1)
    assert (same | band).all() and same.mean() > 0.99
    np.testing.assert_allclose(p[same], r["pdf"][same], rtol=bars.PDF_RTOL)
    del o, g


@pytest.mark.parametrize("N", [16, 32])
def test_guide_pdf_c2(c2, w, torch_dev, N):
    """The frame-scale room at depth 10 with N = 16 (the benchmark's field)
    and N = 32: camera-queue and area-uniform vertices."""
    cam, _ = sample_cols(c2["cam"], 256 if N == 16 else 96, 3)
    rnd, _ = sample_cols(c2["rnd"], 128 if N == 16 else 64, 4)
    _pdf_compare(c2["o"], c2["g"], w, torch_dev, np.concatenate([cam, rnd], 1), N, c2["C"],
                 name="guide_pdf C2")


@pytest.mark.parametrize("fmt", [1, 2])
def test_guide_pdf_16bit_storage(orc, w, torch_dev, c1, fmt):
    """16-bit exitance and bins: within 2e-3 of the oracle fed the same
    quantized values (the oracle rounds exactly as the kernels store, so the
    FP32-path bar of 1e-5 is kept), and the error against the FP64 field is
    reported."""
    box = c1["rects"]
    o = orc.SVO(box, 6)
    o.accumulate(*c1["splats"])
    o.propagate(fmt)
    g = w.svo_build(box, 6, fmt)
    w.svo_accumulate(g, *to_dev(torch_dev, *c1["splats"]))
    pos = c1["pos"][:, :1024]
    (dpos,) = to_dev(torch_dev, pos)
    got = w.guide_pdf(g, dpos, w.make_opts(N=8)).cpu().numpy().astype(np.float64)
    want, truth = o.guide_pdf(pos, 8, truth=True)
    rel = np.abs(got - want) / want
    bars.record(f"guide_pdf C1 fmt{fmt} N=8 rel", rel.max(), bars.pdf_bound(8))
    assert rel.max() <= bars.PDF_RTOL
    err_truth = np.abs(got - truth) / truth
    print(f"fmt {fmt}: max rel err vs FP64 field {err_truth.max():.3e}, mean {err_truth.mean():.3e}")
    assert err_truth.max() < 2e-2


@pytest.fixture(scope="module", params=[1, 2], ids=["fp16", "bf16"])
def c4(request, orc, w, torch_dev):
    """The frame-scale room at depth 10 with 16-bit exitance storage, one
    splat per (leaf, side) so that the stored values do not depend on the
    order of the atomic additions: the oracle stores exactly what the
    kernels store."""
    fmt = request.param
    room = synth.room()
    o = orc.SVO(room, 10)
    xyz, em = o.leaf_info()
    sp = synth.leaf_splats(xyz, o.normals(10), em, 10, seed=22)
    assert o.accumulate(*sp) == 0
    o.propagate(fmt)
    g = w.svo_build(room, 10, fmt)
    w.svo_accumulate(g, *to_dev(torch_dev, *sp))
    cam, _, _ = synth.camera_queue(room)
    rnd, _, _ = synth.area_points(room, 4096, 24)
    pos = np.ascontiguousarray(np.concatenate([cam[:, ::4051], rnd[:, :256]], 1))
    yield dict(fmt=fmt, o=o, g=g, pos=pos)
    del g


def test_guide_pdf_c4_room(c4, w, torch_dev):
    """Exitance and bins stored in FP16 / BF16 on the frame-scale room, N = 16:
    the pdf within the FP32 bar of the oracle fed the same 16-bit values (2e-3
    is the stated bar of the reduced form; the inputs being identical, the
    FP32 one holds), and the error against the unquantized FP64 field
    recorded."""
    want, truth = c4["o"].guide_pdf(c4["pos"], 16, truth=True)
    rel = _pdf_compare(c4["o"], c4["g"], w, torch_dev, c4["pos"], 16, name=f"guide_pdf C4 fmt{c4['fmt']}",
                       want=want)
    assert rel <= 2e-3
    (dpos,) = to_dev(torch_dev, c4["pos"])
    got = w.guide_pdf(c4["g"], dpos, w.make_opts(N=16)).cpu().numpy().astype(np.float64)
    err = np.abs(got - truth) / truth
    bars.record(f"guide_pdf C4 fmt{c4['fmt']} vs FP64 field (reported)", err.max())
    assert err.max() < 2e-2


def test_guide_sample_c4_room(orc, c4, w, torch_dev):
    """guide_sample with 16-bit storage on the frame-scale room, N = 16,
    against the oracle fed the same 16-bit values, at the FP32 sampling bars."""
    _sample_compare(orc, c4["o"], c4["g"], w, torch_dev, c4["pos"], 16, seed=91, bounce=0,
                    name=f"guide_sample C4 fmt{c4['fmt']}")


# ----------------------------------------------------------- guide_sample ----
def _sample_compare(orc, o, g, w, torch_dev, pos, N, seed, bounce, C=1, name="sample", ref=None,
                    got=None):
    if got is None:
        (dpos,) = to_dev(torch_dev, pos)
        d, p = w.guide_sample(g, dpos, w.make_opts(N=N), seed=seed, bounce=bounce)
    else:
        d, p = got
    d = d.cpu().numpy().astype(np.float64)
    p = p.cpu().numpy().astype(np.float64)
    if ref is None:
        ref = o.guide_sample(pos, N, seed=seed, bounce=bounce)
    BAND, EDGE = bars.scan_band(N, C), bars.edge_band(N)
    xy = orc.oct_encode_many(d)
    gb = np.stack([np.minimum((xy[0] * N).astype(int), N - 1),
                   np.minimum((xy[1] * N).astype(int), N - 1)], 1)
    fx, fy = xy[0] * N, xy[1] * N
    edge = np.minimum(np.abs(fx - np.rint(fx)), np.abs(fy - np.rint(fy)))
    same = (gb == ref["bin"]).all(1)
    band = ref["margin"].min(1) < BAND
    bad = ~same & ~band & (edge > EDGE)
    assert not bad.any(), np.nonzero(bad)[0][:10]
    assert same.mean() > 0.99
    ok = same & (edge > EDGE)
    a_ = d[:, ok] / np.linalg.norm(d[:, ok], axis=0)
    b_ = ref["dir"][:, ok]
    ang = 2 * np.arcsin(np.minimum(np.linalg.norm(a_ - b_, axis=0) / 2, 1.0))
    bars.record(f"{name} N={N} dir", ang.max(), bars.DIR_TOL)
    assert ang.max() < bars.DIR_TOL, ang.max()
    rel = np.abs(p[same] - ref["pdf"][same]) / ref["pdf"][same]
    bars.record(f"{name} N={N} rel", rel.max(), bars.pdf_bound(N, C))
    assert rel.max() <= bars.PDF_RTOL
    np.testing.assert_allclose(np.linalg.norm(d, axis=0), 1.0, atol=2e-6)
    return (~same).sum()


def test_guide_sample_c1(orc, c1, w, torch_dev):
    for N in (8, 16, 32):
        _sample_compare(orc, c1["o"], c1["g"], w, torch_dev, c1["pos"], N, seed=11 + N, bounce=2,
                        name="guide_sample C1")


@pytest.mark.parametrize("N", [16, 32])
def test_guide_sample_c2(orc, c2, w, torch_dev, N):
    cam, _ = sample_cols(c2["cam"], 512 if N == 16 else 192, 5)
    rnd, _ = sample_cols(c2["rnd"], 128, 6)
    _sample_compare(orc, c2["o"], c2["g"], w, torch_dev, np.concatenate([cam, rnd], 1), N, seed=123 + N,
                    bounce=0, C=c2["C"], name="guide_sample C2")


def test_sample_chi2_gpu(orc, c1, w, torch_dev):
    from scipy import stats
    torch, dev = torch_dev
    N = 8
    n = 1 << 20
    o, g = c1["o"], c1["g"]
    for vi in (0, 1):
        pos = np.repeat(c1["pos"][:, vi:vi + 1], n, 1)
        (dpos,) = to_dev(torch_dev, pos)
        d, _ = w.guide_sample(g, dpos, w.make_opts(N=N), seed=77 + vi, bounce=1)
        xy = orc.oct_encode_many(d.cpu().numpy().astype(np.float64))
        b = np.minimum((xy[1] * N).astype(int), N - 1) * N + np.minimum((xy[0] * N).astype(int), N - 1)
        h = np.bincount(b, minlength=N * N).astype(float)
        prob = o.guide_pdf(c1["pos"][:, vi:vi + 1], N)[0] * 4 * math.pi / N ** 2
        e = prob * n
        keep = e >= 5
        hs = np.append(h[keep], h[~keep].sum())
        es = np.append(e[keep], e[~keep].sum())
        if es[-1] == 0:
            hs, es = hs[:-1], es[:-1]
        assert stats.chisquare(hs, es).pvalue > 1e-3


# --------------------------------------------------------------- pdf_eval ----
def test_pdf_eval_c1(orc, c1, w, torch_dev):
    o, g = c1["o"], c1["g"]
    pos = c1["pos"][:, :2048]
    rng = np.random.default_rng(8)
    v = rng.normal(size=(3, pos.shape[1]))
    v = (v / np.linalg.norm(v, axis=0)).astype(np.float32)
    for N in (8, 16):
        dpos, dv = to_dev(torch_dev, pos, v)
        got = w.pdf_eval(g, dpos, dv, w.make_opts(N=N)).cpu().numpy().astype(np.float64)
        ref = o.pdf_eval(pos, v, N)
        ok = ref["edge"] > bars.edge_band(N)
        assert ok.mean() > 0.99
        rel = np.abs(got[ok] - ref["pdf"][ok]) / ref["pdf"][ok]
        bars.record(f"pdf_eval C1 N={N} rel", rel.max(), bars.pdf_bound(N))
        assert rel.max() <= bars.PDF_RTOL


def test_pdf_eval_c2(orc, c2, w, torch_dev):
    """pdf_eval on the frame-scale room against the oracle's pdf_eval: for
    random directions and for the directions guide_sample returned (which
    lie anywhere inside their bins); the bin may differ only within the
    encode band of a bin edge."""
    torch, dev = torch_dev
    cam, _ = sample_cols(c2["cam"], 2048, 9)
    (dpos,) = to_dev(torch_dev, cam)
    opts = w.make_opts(N=16)
    d, p = w.guide_sample(c2["g"], dpos, opts, seed=5, bounce=1)
    rng = np.random.default_rng(10)
    v = rng.normal(size=(3, cam.shape[1]))
    v = (v / np.linalg.norm(v, axis=0)).astype(np.float32)
    for dirs in (d.cpu().numpy(), v):
        got = w.pdf_eval(c2["g"], dpos, to_dev(torch_dev, dirs)[0], opts).cpu().numpy().astype(np.float64)
        ref = c2["o"].pdf_eval(cam, dirs, 16)
        ok = ref["edge"] > bars.edge_band(16)
        assert ok.mean() > 0.99
        rel = np.abs(got[ok] - ref["pdf"][ok]) / ref["pdf"][ok]
        bars.record("pdf_eval C2 N=16 rel", rel.max(), bars.pdf_bound(16, c2["C"]))
        assert rel.max() <= bars.PDF_RTOL
    # and the sampler's own pdf is what pdf_eval returns for its direction
    q = w.pdf_eval(c2["g"], dpos, d, opts)
    agree = (torch.abs(p - q) <= 1e-6 * p).float().mean().item()
    assert agree > 0.999


# -------------------------------------------------------------- edge cases ---
def test_edge_cases(orc, w, torch_dev, c1):
    torch, dev = torch_dev
    g = c1["g"]
    opts = w.make_opts(N=8)
    empty = torch.empty((3, 0), device=dev)
    w.guide_sample(g, empty, opts, 1, 0)
    w.guide_pdf(g, empty, opts)
    w.svo_accumulate(g, empty, empty, empty)  # recomputes averages only
    # ragged queue lengths (not multiples of the waves of a block)
    for n in (1, 3, 63, 65, 1001):
        pos = c1["pos"][:, :n]
        (dpos,) = to_dev(torch_dev, pos)
        got = w.guide_pdf(g, dpos, opts).cpu().numpy()
        want = c1["o"].guide_pdf(pos, 8)
        assert (np.abs(got - want) / want).max() <= bars.PDF_RTOL
    # invalid arguments
    bad = w.make_opts(N=12)
    with pytest.raises(w.WfpgError):
        w.guide_pdf(g, to_dev(torch_dev, c1["pos"][:, :4])[0], bad)
    with pytest.raises(w.WfpgError) as ei:
        w.guide_sample(g, to_dev(torch_dev, c1["pos"][:, :4])[0], w.make_opts(N=8, mode=1), 1, 0)
    assert ei.value.status == -4
    with pytest.raises(w.WfpgError):
        w.guide_pdf(g, to_dev(torch_dev, c1["pos"][:, :4])[0], w.make_opts(N=8, eps=0.0))


def test_empty_svo_all_miss(w, torch_dev):
    torch, dev = torch_dev
    g = w.svo_build(np.zeros(0, synth.RECT_DTYPE), 5)
    assert g.level_sizes() == [0] * 6
    pos = torch.rand((3, 100), device=dev)
    pdf = w.guide_pdf(g, pos, w.make_opts(N=16))
    assert torch.allclose(pdf, torch.full_like(pdf, 1 / (4 * math.pi)), rtol=1e-6)
    sp = torch.rand((3, 10), device=dev)
    w.svo_accumulate(g, sp, sp, sp)
    assert g.stats()["dropped"] == 10


def test_invalid_splats_dropped(orc, w, torch_dev):
    torch, dev = torch_dev
    box = synth.cornell_box()
    o = orc.SVO(box, 6)
    g = w.svo_build(box, 6)
    pos, nrm, _ = synth.area_points(box, 1000, 4)
    rgb = np.ones((3, 1000), np.float32)
    pos[0, 0] = np.nan
    pos[1, 1] = 1.5
    rgb[2, 2] = np.inf
    rgb[:, 3] = -1.0
    pos[:, 5] = 0.5
    nd = o.accumulate(pos, nrm, rgb)
    w.svo_accumulate(g, *to_dev(torch_dev, pos, nrm, rgb))
    assert g.stats()["dropped"] == nd == 5
    s, c = g.export_accum()
    _, _, oc = o.leaf_accum()
    assert np.array_equal(c.astype(np.int64), oc)


def test_uniform_enclosure_gpu(w, torch_dev):
    """Closed box, every splat 1.0 on both sides: every inner node averages
    to 1.0 and an interior point sees the uniform pdf 1/(4 pi)."""
    torch, dev = torch_dev
    rs = []
    for a in range(3):
        rs.append(synth.make_rect(a, 0.0, (0, 0), (1, 1), +1))
        rs.append(synth.make_rect(a, 1.0, (0, 0), (1, 1), -1))
    rs = np.array(rs, synth.RECT_DTYPE)
    g = w.svo_build(rs, 5)
    keys, nrm, _ = g.export_level(5)
    xyz = np.stack([np.array([sum(((int(k) >> (3 * i + a)) & 1) << i for i in range(5)) for k in keys])
                    for a in range(3)], 1)
    sp = synth.leaf_splats(xyz, nrm, np.zeros(len(keys)), 5)
    ones = np.ones_like(sp[2])
    w.svo_accumulate(g, *to_dev(torch_dev, sp[0], sp[1], ones))
    for l in range(6):
        _, _, ex = g.export_level(l)
        assert (ex == 1.0).all()
    pos = torch.rand((3, 64), device=dev) * 0.8 + 0.1
    pdf = w.guide_pdf(g, pos, w.make_opts(N=16))
    assert torch.allclose(pdf, torch.full_like(pdf, 1 / (4 * math.pi)), rtol=1e-6)


# ------------------------------------------------- full size, bench launch ---
def test_full_size_headline_queue(orc, c2, w, torch_dev):
    """guide_sample over the whole 1920x1080 camera queue in the benchmark's
    launch configuration; every 1013th vertex checked against the oracle."""
    torch, dev = torch_dev
    cam = c2["cam"]
    (dpos,) = to_dev(torch_dev, cam)
    opts = w.make_opts(N=16)
    d, p = w.guide_sample(c2["g"], dpos, opts, seed=2024, bounce=0)
    d2, p2 = w.guide_sample(c2["g"], dpos, opts, seed=2024, bounce=0)
    assert torch.equal(d, d2) and torch.equal(p, p2)   # deterministic
    assert torch.isfinite(p).all() and (p > 0).all()
    assert torch.allclose(torch.linalg.norm(d, dim=0), torch.ones_like(p), atol=2e-6)
    idx = np.arange(0, cam.shape[1], 1013)
    sub = np.ascontiguousarray(cam[:, idx])
    ref = c2["o"].guide_sample(sub, 16, seed=2024, bounce=0, counter=idx)
    gd = d.cpu().numpy()[:, idx].astype(np.float64)
    gp = p.cpu().numpy()[idx].astype(np.float64)
    xy = orc.oct_encode_many(gd)
    gb = np.stack([np.minimum((xy[0] * 16).astype(int), 15), np.minimum((xy[1] * 16).astype(int), 15)], 1)
    same = (gb == ref["bin"]).all(1)
    fx, fy = xy[0] * 16, xy[1] * 16
    edge = np.minimum(np.abs(fx - np.rint(fx)), np.abs(fy - np.rint(fy)))
    band, eb = bars.scan_band(16, c2["C"]), bars.edge_band(16)
    assert not (~same & (ref["margin"].min(1) >= band) & (edge > eb)).any()
    rel = np.abs(gp[same] - ref["pdf"][same]) / ref["pdf"][same]
    bars.record("guide_sample full queue N=16 rel", rel.max(), bars.pdf_bound(16, c2["C"]))
    assert same.mean() > 0.99 and rel.max() <= bars.PDF_RTOL
    assert g_stats_ok(c2["g"])


def g_stats_ok(g):
    return g.stats()["errors"] == 0
