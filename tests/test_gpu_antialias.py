"""GPU parity of the field antialiasing options (Sec. 4: directional jitter and
Gaussian blur) through the C ABI, against the oracle: the jittered cone
directions bit for bit, and guide_pdf / guide_sample / pdf_eval, the binned
fields and the product sampler with the options on, at the FP32 bars of the
plain paths (pdf within 1e-5 relative; sampled bins equal outside the scan
band; directions within 2e-6; the bars are derived in tests/bars.py).
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
    out = {}
    for fmt in (0, 2):
        o = orc.SVO(rects, D)
        xyz, em = o.leaf_info()
        sp = synth.leaf_splats(xyz, o.normals(D), em, D, seed=2)
        assert o.accumulate(*sp) == 0
        o.propagate(fmt)
        g = w.svo_build(rects, D, fmt)
        w.svo_accumulate(g, *[dev(torch_dev, a) for a in sp])
        out[fmt] = (o, g)
    pos, nrm, _ = synth.area_points(rects, 1500, 11)
    extra = np.random.default_rng(3).uniform(0.3, 0.7, (3, 29)).astype(np.float32)
    pos = np.ascontiguousarray(np.concatenate([pos, extra], 1))
    nrm = np.ascontiguousarray(np.concatenate([nrm, np.tile([[0.0], [0.0], [1.0]], (1, 29)).astype(np.float32)], 1))
    return dict(svo=out, pos=pos, nrm=nrm)


@pytest.mark.parametrize("N", [8, 16, 32, 64, 128])
def test_jitter_table_bitexact(w, N):
    for key in (0, 1, 2024, 0xFFFFFFFF):
        got = w.dir_table_jitter(N, key)
        want = oracle.jitter_table(N, key)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (N, key)


CASES = [(8, 7, False), (16, 7, False), (16, None, True), (32, 99, True)]


@pytest.mark.parametrize("fmt", [0, 2])
@pytest.mark.parametrize("N,key,blur", CASES)
def test_guide_pdf_antialiased(c1, w, torch_dev, fmt, N, key, blur):
    o, g = c1["svo"][fmt]
    pos = c1["pos"]
    got = w.guide_pdf(g, dev(torch_dev, pos), w.make_opts(N=N, jitter_key=key, blur=blur)).cpu().numpy()
    L = o.field_aa(pos, N, jitter_key=key, blur=blur)
    want = L / L.sum(1, keepdims=True) * (N * N) / (4 * np.pi)
    rel = np.abs(got - want) / want   # the oracle rounds as the kernels store
    bars.record(f"antialiased guide_pdf N={N} rel", rel.max(), bars.pdf_bound(N))
    assert rel.max() <= bars.PDF_RTOL
    if key is not None:   # the options change the field
        plain = w.guide_pdf(g, dev(torch_dev, pos), w.make_opts(N=N)).cpu().numpy()
        assert not np.array_equal(plain, got)


def check_samples(d, p, r, N, seq=False, name="antialiased"):
    """seq: the sampler's CDFs are sequential prefix sums (binned, product)."""
    d, p = d.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64)
    uv = oracle.oct_encode_many(d)
    gb = np.minimum((uv * N).astype(np.int64), N - 1)
    same = (gb[0] == r["bin"][:, 0]) & (gb[1] == r["bin"][:, 1])
    band = (r["margin"] < (bars.scan_band_seq(N) if seq else bars.scan_band(N))).any(1)
    assert (same | band).all(), np.nonzero(~(same | band))[0][:10]
    assert same.mean() > 0.999
    rel = np.abs(p[same] - r["pdf"][same]) / r["pdf"][same]
    bars.record(f"{name} N={N} rel", rel.max())
    assert rel.max() <= bars.PDF_RTOL
    chord = np.linalg.norm(d[:, same] - r["dir"][:, same], axis=0)
    bars.record(f"{name} N={N} dir", chord.max(), bars.DIR_TOL)
    assert chord.max() < bars.DIR_TOL, chord.max()
    return d, p


@pytest.mark.parametrize("N,key,blur", CASES)
def test_guide_sample_and_eval_antialiased(c1, w, torch_dev, N, key, blur):
    o, g = c1["svo"][0]
    pos = c1["pos"]
    opts = w.make_opts(N=N, jitter_key=key, blur=blur)
    d, p = w.guide_sample(g, dev(torch_dev, pos), opts, 13, 2)
    L = o.field_aa(pos, N, jitter_key=key, blur=blur)
    r = oracle.sample_fields(L, N, 13, 2)
    d, p = check_samples(d, p, r, N)
    pe = w.pdf_eval(g, dev(torch_dev, pos), dev(torch_dev, d.astype(np.float32)), opts).cpu().numpy()
    uv = oracle.oct_encode_many(d)
    ok = np.abs(uv * N - np.rint(uv * N)).min(0) > bars.edge_band(N)
    assert np.array_equal(pe[ok], p.astype(np.float32)[ok])


@pytest.mark.parametrize("N,c_ray,l_min,key,blur", [(8, 64, 3, 5, True), (16, 64, 3, 5, True),
                                                    (32, 256, 2, None, True), (64, 256, 2, 8, False),
                                                    (128, 1024, 1, 8, True)])
def test_binned_antialiased(c1, w, torch_dev, N, c_ray, l_min, key, blur):
    o, g = c1["svo"][0]
    pos = c1["pos"]
    d, p = w.guide_sample_binned(g, dev(torch_dev, pos),
                                 w.bin_opts(N=N, c_ray=c_ray, l_min=l_min, jitter_key=key, blur=blur), 21, 2)
    r = o.binned_sample(pos, c_ray, l_min, N, 21, 2, jitter_key=key, blur=blur)
    check_samples(d, p, r, N, seq=True, name="antialiased binned")


@pytest.mark.parametrize("N", [16, 32])
def test_product_antialiased(c1, w, torch_dev, N):
    o, g = c1["svo"][0]
    pos, nrm = c1["pos"], c1["nrm"]
    opts = w.make_opts(N=N, jitter_key=41, blur=True)
    d, p = w.guide_sample_product(g, dev(torch_dev, pos), opts, 3, 1, nrm=dev(torch_dev, nrm))
    L = o.field_aa(pos, N, jitter_key=41, blur=True)
    r = oracle.product_sample_fields(L, N, 3, 1, nrm=nrm)
    check_samples(d, p, r, N, seq=True, name="antialiased product")
    d2, p2 = w.guide_sample_binned_product(g, dev(torch_dev, pos),
                                           w.bin_opts(N=N, c_ray=64, l_min=3, jitter_key=41, blur=True), 3, 1,
                                           nrm=dev(torch_dev, nrm))
    r2 = o.binned_sample(pos, 64, 3, N, 3, 1, nrm=nrm, jitter_key=41, blur=True)
    check_samples(d2, p2, r2, N, seq=True, name="antialiased binned product")


def test_antialias_errors(c1, w, torch_dev):
    _, g = c1["svo"][0]
    pos = dev(torch_dev, c1["pos"])
    bad = w.Opts(16, 0.01, 0, 0.05, 256, 2, 0, 0)
    with pytest.raises(w.WfpgError):
        w.guide_pdf(g, pos, bad)
    with pytest.raises(w.WfpgError):
        w.guide_sample_binned(g, pos, w.BinOpts(16, 0.01, 64, 3, 0, 0, 3), 0, 0)
