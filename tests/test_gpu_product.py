"""GPU parity of product path guiding (Sec. 3.6) through the C ABI, against the
oracle: the per-vertex product sampler and pdf (guide_sample_product,
pdf_eval_product) and the binned product sampler
(guide_sample_binned_product).

Bars: sampled fine bins equal to the oracle's outside the FP32 scan band at
CDF boundaries of either level; pdfs within 1e-5 relative of the oracle's
FP64 values; directions within 2e-6 (chord) of the oracle's FP64 decode; the
GPU's own pdf_eval_product bit-identical to the pdf it returned for a sample.
"""
import numpy as np
import pytest

import oracle
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
    pos, nrm, _ = synth.area_points(rects, 3000, 3)
    rng = np.random.default_rng(8)
    extra = rng.uniform(0.3, 0.7, (3, 37)).astype(np.float32)       # ragged, off-surface
    en = rng.normal(size=(3, 37)).astype(np.float32)
    en[:, :3] = 0.0                                                  # degenerate normals: plain guiding
    pos = np.ascontiguousarray(np.concatenate([pos, extra], 1))
    nrm = np.ascontiguousarray(np.concatenate([nrm, en], 1))
    tab = rng.uniform(-0.2, 1.0, (pos.shape[1], 64)).astype(np.float32)   # some entries clip to 0
    return dict(o=o, g=g, pos=pos, nrm=nrm, tab=tab)


def check_samples(d, p, r, N):
    d, p = d.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64)
    uv = oracle.oct_encode_many(d)
    gb = np.minimum((uv * N).astype(np.int64), N - 1)
    same = (gb[0] == r["bin"][:, 0]) & (gb[1] == r["bin"][:, 1])
    band = (r["margin"] < bars.scan_band_seq(N)).any(1)
    assert (same | band).all(), np.nonzero(~(same | band))[0][:10]
    assert same.mean() > 0.999
    rel = np.abs(p[same] - r["pdf"][same]) / r["pdf"][same]
    bars.record(f"product N={N} rel", rel.max())
    assert rel.max() <= bars.PDF_RTOL
    chord = np.linalg.norm(d[:, same] - r["dir"][:, same], axis=0)
    bars.record(f"product N={N} dir", chord.max(), bars.DIR_TOL)
    assert chord.max() < bars.DIR_TOL, chord.max()
    return d, p


@pytest.mark.parametrize("N", [8, 16, 32])
@pytest.mark.parametrize("table", ["nrm", "bsdf"])
def test_product_sample_matches_oracle(c1, w, torch_dev, N, table):
    o, g, pos = c1["o"], c1["g"], c1["pos"]
    kw = dict(nrm=c1["nrm"]) if table == "nrm" else dict(bsdf=c1["tab"])
    seed, bounce = 17, 3
    opts = w.make_opts(N=N)
    d, p = w.guide_sample_product(g, dev(torch_dev, pos), opts, seed, bounce,
                                  **{k: dev(torch_dev, v) for k, v in kw.items()})
    r = o.product_sample(pos, N, seed, bounce, **kw)
    d, p = check_samples(d, p, r, N)
    # the GPU's own pdf of its samples: bit-identical
    dd = dev(torch_dev, d.astype(np.float32))
    pe = w.pdf_eval_product(g, dev(torch_dev, pos), dd, opts, **{k: dev(torch_dev, v) for k, v in kw.items()})
    uv = oracle.oct_encode_many(d)
    edge = np.abs(uv * N - np.rint(uv * N)).min(0)
    ok = edge > bars.edge_band(N)
    assert np.array_equal(pe.cpu().numpy()[ok], p.astype(np.float32)[ok])


@pytest.mark.parametrize("N", [8, 16, 32])
def test_pdf_eval_product_matches_oracle(c1, w, torch_dev, N):
    o, g, pos, nrm = c1["o"], c1["g"], c1["pos"], c1["nrm"]
    dirs = np.random.default_rng(N).normal(size=pos.shape)
    dirs = (dirs / np.linalg.norm(dirs, axis=0)).astype(np.float32)
    pe = w.pdf_eval_product(g, dev(torch_dev, pos), dev(torch_dev, dirs), w.make_opts(N=N),
                            nrm=dev(torch_dev, nrm)).cpu().numpy()
    r = o.product_pdf_eval(pos, dirs, N, nrm=nrm)
    ok = r["edge"] > bars.edge_band(N)
    np.testing.assert_allclose(pe[ok], r["pdf"][ok], rtol=bars.PDF_RTOL)


def test_product_chi_square_one_vertex(c1, w, torch_dev):
    """2^20 queries at one vertex: the GPU's samples follow the direct product
    definition (fine field times the cell-constant table, normalized)."""
    from scipy.stats import chi2
    o, g = c1["o"], c1["g"]
    N, n = 16, 1 << 20
    p0, n0 = c1["pos"][:, 5:6], c1["nrm"][:, 5:6]
    pos = np.ascontiguousarray(np.repeat(p0, n, 1))
    nrm = np.ascontiguousarray(np.repeat(n0, n, 1))
    d, _ = w.guide_sample_product(g, dev(torch_dev, pos), w.make_opts(N=N), 5, 0, nrm=dev(torch_dev, nrm))
    uv = oracle.oct_encode_many(d.cpu().numpy().astype(np.float64))
    b = np.minimum((uv * N).astype(np.int64), N - 1)
    cnt = np.bincount(b[1] * N + b[0], minlength=N * N)
    L, _ = o.field(p0, N)
    dt = oracle.dir_table(8).reshape(64, 3).astype(np.float32)
    nn = n0[:, 0].astype(np.float32)
    cos = (nn[0] * dt[:, 0] + nn[1] * dt[:, 1]) + nn[2] * dt[:, 2]
    f = np.where(cos > 0, cos, 0).astype(np.float64)
    fu = np.kron(f.reshape(8, 8), np.ones((2, 2))).reshape(N * N)
    prob = L[0] * fu / (L[0] * fu).sum()
    assert cnt[prob == 0].sum() == 0
    exp = prob * n
    big = exp >= 5
    stat = (((cnt[big] - exp[big]) ** 2) / exp[big]).sum()
    dof = big.sum() - 1
    assert chi2.sf(stat, dof) > 1e-4


@pytest.mark.parametrize("N,c_ray,l_min", [(8, 64, 3), (16, 64, 3), (32, 256, 2), (64, 256, 2), (128, 1024, 1)])
def test_binned_product_matches_oracle(c1, w, torch_dev, N, c_ray, l_min):
    o, g, pos, nrm = c1["o"], c1["g"], c1["pos"], c1["nrm"]
    seed, bounce = 21, 2
    d, p, b = w.guide_sample_binned_product(g, dev(torch_dev, pos), w.bin_opts(N=N, c_ray=c_ray, l_min=l_min),
                                            seed, bounce, nrm=dev(torch_dev, nrm), bins=True)
    r = o.binned_sample(pos, c_ray, l_min, N, seed, bounce, nrm=nrm)
    sizes = np.array(g.level_sizes(), np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)])
    bb = b.cpu().numpy().astype(np.int64)
    lv = np.searchsorted(off, bb, side="right") - 1
    assert np.array_equal(lv, r["level"]) and np.array_equal(bb - off[lv], r["index"])
    check_samples(d, p, r, N)


def test_binned_product_bsdf_table(c1, w, torch_dev):
    o, g, pos, tab = c1["o"], c1["g"], c1["pos"], c1["tab"]
    d, p = w.guide_sample_binned_product(g, dev(torch_dev, pos), w.bin_opts(N=32, c_ray=128, l_min=3), 4, 1,
                                         bsdf=dev(torch_dev, tab))
    r = o.binned_sample(pos, 128, 3, 32, 4, 1, bsdf=tab)
    check_samples(d, p, r, 32)


def test_product_full_size_queue(orc, w, torch_dev):
    """The frame-scale room and camera queue with the camera-facing normals:
    per-vertex and binned product samples checked on strided vertices."""
    room = synth.room()
    o = orc.SVO(room, 10)
    sp = synth.room_splats(room, 2_000_000, 13)
    o.accumulate(*sp)
    o.propagate()
    g = w.svo_build(room, 10)
    w.svo_accumulate(g, *[dev(torch_dev, a) for a in sp])
    cam, cn, _ = synth.camera_queue(room)
    n = cam.shape[1]
    dpos, dnrm = dev(torch_dev, cam), dev(torch_dev, cn)
    d, p = w.guide_sample_product(g, dpos, w.make_opts(N=16), 6, 0, nrm=dnrm)
    assert (p > 0).all()
    i = np.arange(0, n, n // 512)
    L, _ = o.field(cam[:, i], 16)
    uv = oracle.oct_encode_many(d.cpu().numpy().astype(np.float64)[:, i])
    gb = np.minimum((uv * 16).astype(np.int64), 15)
    frac = uv * 16 - np.floor(uv * 16)
    inner = ((frac > bars.edge_band(16)) & (frac < 1 - bars.edge_band(16))).all(0)
    dt = oracle.dir_table(8).reshape(64, 3).astype(np.float32)
    nn = cn[:, i].astype(np.float32)
    cos = (nn[0][:, None] * dt[None, :, 0] + nn[1][:, None] * dt[None, :, 1]) + nn[2][:, None] * dt[None, :, 2]
    f = np.where(cos > 0, cos, 0).astype(np.float64)
    fu = np.kron(f.reshape(-1, 8, 8), np.ones((1, 2, 2))).reshape(len(i), 256)
    prod = L * fu
    want = (prod / prod.sum(1, keepdims=True) * 256 / (4 * np.pi))[np.arange(len(i)), gb[1] * 16 + gb[0]]
    np.testing.assert_allclose(p.cpu().numpy()[i][inner], want[inner], rtol=bars.PDF_RTOL)
    # binned: every member's pdf is its origin field times its own table at the sampled bin
    d2, p2 = w.guide_sample_binned_product(g, dpos, w.bin_opts(N=16, c_ray=512, l_min=5), 6, 0, nrm=dnrm)
    _, org = w.partition(g, dpos, 512, 5, seed=6, bounce=0)
    orig = org.cpu().numpy()[i]
    Lo, _ = o.field(cam[:, orig], 16)
    uv = oracle.oct_encode_many(d2.cpu().numpy().astype(np.float64)[:, i])
    gb = np.minimum((uv * 16).astype(np.int64), 15)
    frac = uv * 16 - np.floor(uv * 16)
    inner = ((frac > bars.edge_band(16)) & (frac < 1 - bars.edge_band(16))).all(0)
    prod = Lo * fu
    want = (prod / prod.sum(1, keepdims=True) * 256 / (4 * np.pi))[np.arange(len(i)), gb[1] * 16 + gb[0]]
    np.testing.assert_allclose(p2.cpu().numpy()[i][inner], want[inner], rtol=bars.PDF_RTOL)


def test_product_errors(c1, w, torch_dev):
    g, pos = c1["g"], dev(torch_dev, c1["pos"])
    nrm, tab = dev(torch_dev, c1["nrm"]), dev(torch_dev, c1["tab"])
    with pytest.raises(w.WfpgError):
        w.guide_sample_product(g, pos, w.make_opts(N=16), 0, 0)                     # no table
    with pytest.raises(w.WfpgError):
        w.guide_sample_product(g, pos, w.make_opts(N=16), 0, 0, nrm=nrm, bsdf=tab)  # both
    with pytest.raises(w.WfpgError):
        w.guide_sample_product(g, pos, w.make_opts(N=12), 0, 0, nrm=nrm)
    with pytest.raises(w.WfpgError):
        w.guide_sample_binned_product(g, pos, w.bin_opts(N=16, c_ray=64, l_min=3), 0, 0)
    d, p = w.guide_sample_product(g, pos[:, :0].contiguous(), w.make_opts(N=16), 0, 0,
                                  nrm=nrm[:, :0].contiguous())
    assert d.shape == (3, 0)
