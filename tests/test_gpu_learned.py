"""GPU tests of the learned stand-in for the march, through the C ABI.

* The BF16 MFMA forward pass and the backward pass (gradients of the mean
  cross-entropy) agree element by element with the BF16-faithful CPU oracle,
  which rounds to BF16 at the same points (table, inputs, weights, hidden
  activations, logit and pre-activation gradients) but accumulates in FP64.
  The GPU accumulates BF16 products in FP32 inside the matrix cores, in
  another order, so a value within its FP32 accumulation error of a BF16
  rounding boundary may round to the neighbouring BF16 value on one side
  only. The oracle derives, for every probability and every gradient
  element, the bound of the FP32 accumulations plus every such flip they
  allow (tests/test_oracle_nn_bounds.py pins it against an FP32 emulation in
  random orders); the measured errors are recorded against it.
* Sampling from the network returns the pdf of the bin it sampled.
* Training lowers the KL to the march; the judge falls back to the march,
  bit for bit, when the probes' KL exceeds the bound.
"""
import math

import numpy as np
import pytest

import bars
import nn_params
import synth

pytestmark = pytest.mark.gpu

SMALL = dict(log2_table=12, n_min=4, n_max=64)
FOUR_PI = 4 * math.pi


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
def box(w, torch_dev):
    """Cornell box at depth 6 with one exitance splat per (leaf, side) and an
    attached small learned model."""
    import oracle
    rects = synth.cornell_box()
    o = oracle.SVO(rects, 6)
    xyz, em = o.leaf_info()
    sp = synth.leaf_splats(xyz, o.normals(6), em, 6, seed=2)
    assert o.accumulate(*sp) == 0
    o.propagate()
    g = w.svo_build(rects, 6)
    w.svo_accumulate(g, *[dev(torch_dev, a) for a in sp])
    pos, nrm, _ = synth.area_points(rects, 300, 21)
    return dict(rects=rects, g=g, o=o, pos=pos, nrm=nrm)


def small_model(w, torch_dev, rects):
    g = w.svo_build(rects, 6)
    pos, nrm, _ = synth.area_points(rects, 64, 1)
    w.guide_train(g, dev(torch_dev, pos), dev(torch_dev, nrm), steps=0, **SMALL)
    return g


# ------------------------------------------------------------- forward ----
def test_forward_matches_bf16_oracle(orc, w, torch_dev, box):
    """Every probability within the oracle's derived bound of the
    BF16-faithful forward (FP32 accumulation plus every BF16 flip it allows,
    propagated to the logits and through the softmax)."""
    cfg = orc.nn_cfg(**SMALL)
    n_par = orc.nn_num_params(cfg)
    g = small_model(w, torch_dev, box["rects"])
    assert w.nn_param_count(g) == n_par
    params = nn_params.random_params(n_par, np.random.default_rng(3))
    w.nn_set_params(g, params)
    assert np.array_equal(w.nn_get_params(g), params)
    pos, nrm = box["pos"], box["nrm"]          # 300 rows: 4 full 64-row tiles and a ragged one
    prob = w.nn_forward(g, dev(torch_dev, pos), dev(torch_dev, nrm)).cpu().numpy().astype(np.float64)
    p1, _ = orc.nn_forward(params, cfg, pos, nrm, mode=1)
    pe, _ = orc.nn_parity_bounds(params, cfg, pos, nrm)
    assert np.allclose(prob.sum(1), 1, atol=1e-5)
    rel = np.abs(prob - p1) / p1
    bars.record("nn forward rel (median)", np.median(rel))
    bars.record("nn forward rel / bound", (rel / pe).max(), 1.0)
    bars.record("nn forward rel", rel.max(), 1e-3)
    assert (rel <= pe).all(), (rel / pe).max()
    kl_gpu = orc.kl_rows(p1, prob)
    assert kl_gpu.max() < 1e-5, kl_gpu.max()


def test_forward_pinned_structure(orc, w, torch_dev, box):
    """Zero output layer: exactly uniform; zero MLP except the output bias:
    exactly softmax(b4) at every vertex."""
    cfg = orc.nn_cfg(**SMALL)
    n_par = orc.nn_num_params(cfg)
    g = small_model(w, torch_dev, box["rects"])
    params = nn_params.random_params(n_par, np.random.default_rng(4))
    lay = nn_params.layout(n_par)
    for name in ("W4", "b4"):
        a, m = lay[name]
        params[a:a + m] = 0
    w.nn_set_params(g, params)
    pos, nrm = dev(torch_dev, box["pos"]), dev(torch_dev, box["nrm"])
    prob = w.nn_forward(g, pos, nrm).cpu().numpy()
    assert (prob == np.float32(1 / 256)).all()
    a, m = lay["b4"]
    b4 = np.random.default_rng(5).normal(0, 2, m).astype(np.float32)
    params[a:a + m] = b4
    a, m = lay["W4"]
    params[a:a + m] = 0
    w.nn_set_params(g, params)
    prob = w.nn_forward(g, pos, nrm).cpu().numpy()
    want = np.exp(b4.astype(np.float64) - b4.max())
    want /= want.sum()
    np.testing.assert_allclose(prob, np.broadcast_to(want, prob.shape), rtol=2e-6)


# ------------------------------------------------------------ backward ----
def test_gradient_matches_bf16_oracle(orc, w, torch_dev, box):
    """Every gradient element within the oracle's derived bound around the
    BF16-faithful gradient: FP32 accumulation over the rows and within the
    products, plus every BF16 flip the accumulations allow (forward
    activations, logit and hidden gradients, ReLU masks), propagated as
    intervals. The bound is tight at the output layer and loose towards the
    input, where worst-case flips compound; the per-block norms of the
    difference are therefore also held against the whole BF16 rounding
    effect, which a dropped term or a transposed operand exceeds by far."""
    cfg = orc.nn_cfg(**SMALL)
    n_par = orc.nn_num_params(cfg)
    g = small_model(w, torch_dev, box["rects"])
    rng = np.random.default_rng(6)
    params = nn_params.random_params(n_par, rng)
    w.nn_set_params(g, params)
    B = 256   # rows; a power of two, so the batch scale 1/B is exact in FP32
    pos, nrm = np.ascontiguousarray(box["pos"][:, :B]), np.ascontiguousarray(box["nrm"][:, :B])
    t32 = (rng.random((B, 256)) ** 4).astype(np.float32)
    t32 /= t32.sum(1, keepdims=True)
    t = t32.astype(np.float64)
    t /= t.sum(1, keepdims=True)             # the kernels renormalize the target rows in FP32
    loss, grad = w.nn_grad(g, dev(torch_dev, pos), dev(torch_dev, nrm), dev(torch_dev, t32))
    grad = grad.cpu().numpy().astype(np.float64)
    l1, g1 = orc.nn_grad(params, cfg, pos, nrm, t, mode=1)
    l0, g0 = orc.nn_grad(params, cfg, pos, nrm, t, mode=0)
    _, gr = orc.nn_parity_bounds(params, cfg, pos, nrm, target=t, inv_b=1.0 / B)
    assert abs(loss - l1) < 1e-5 * abs(l1), (loss, l1)
    d = np.abs(grad - g1)
    bars.record("nn gradient |diff| / bound", (d / np.maximum(gr, 1e-300)).max(), 1.0)
    assert (d <= gr * (1 + 1e-9) + 1e-300).all(), (d / np.maximum(gr, 1e-300)).max()
    lay = nn_params.layout(n_par)
    for name, (a, m) in lay.items():
        gg, ref = g1[a:a + m], g0[a:a + m]
        big = np.abs(gg) > 1e-3 * np.abs(gg).max()
        rel = d[a:a + m][big] / np.abs(gg[big])
        bars.record(f"nn gradient {name} rel (median)", np.median(rel), 1e-3)
        bars.record(f"nn gradient {name} rel (max)", rel.max())
        bars.record(f"nn gradient {name} bound rel (median)", np.median(gr[a:a + m][big] / np.abs(gg[big])))
        assert np.median(rel) <= 1e-3, (name, np.median(rel))   # the typical element: no flip reaches it
        nd = np.linalg.norm(d[a:a + m])
        nref = np.linalg.norm(ref - gg)
        assert nd <= 0.5 * nref + 1e-6 * np.linalg.norm(gg), (name, nd, nref)
    # the table gradient touches exactly the corners of the encoded cells
    a, m = lay["table"]
    assert np.array_equal(grad[a:a + m] != 0, g1[a:a + m] != 0)


def test_gradient_step_descends(orc, w, torch_dev, box):
    """One small step against the GPU gradient lowers the FP64 oracle's loss by
    about |g|^2 * lr (first order)."""
    cfg = orc.nn_cfg(**SMALL)
    n_par = orc.nn_num_params(cfg)
    g = small_model(w, torch_dev, box["rects"])
    rng = np.random.default_rng(7)
    params = nn_params.random_params(n_par, rng)
    w.nn_set_params(g, params)
    pos, nrm = box["pos"], box["nrm"]
    t = rng.random((pos.shape[1], 256)) ** 4
    t /= t.sum(1, keepdims=True)
    _, grad = w.nn_grad(g, dev(torch_dev, pos), dev(torch_dev, nrm), dev(torch_dev, t.astype(np.float32)))
    grad = grad.cpu().numpy().astype(np.float64)
    l0, _ = orc.nn_grad(params, cfg, pos, nrm, t, mode=0)
    lr = 1e-3 / np.linalg.norm(grad)
    l1, _ = orc.nn_grad((params - lr * grad).astype(np.float32), cfg, pos, nrm, t, mode=0)
    want = lr * np.dot(grad, grad)
    assert 0.5 * want < l0 - l1 < 1.5 * want, (l0 - l1, want)


# ------------------------------------------------------------ sampling ----
def test_learned_sample_returns_pdf_of_sampled_bin(orc, w, torch_dev, box):
    cfg = orc.nn_cfg(**SMALL)
    n_par = orc.nn_num_params(cfg)
    g = small_model(w, torch_dev, box["rects"])
    params = nn_params.random_params(n_par, np.random.default_rng(8))
    w.nn_set_params(g, params)
    pos, nrm = box["pos"], box["nrm"]
    dpos, dnrm = dev(torch_dev, pos), dev(torch_dev, nrm)
    prob = w.nn_forward(g, dpos, dnrm).cpu().numpy().astype(np.float64)
    opts = w.make_opts(N=16, mode=1, kl_bound=1e30, probe_stride=7)
    d, pdf = w.guide_sample(g, dpos, opts, seed=11, bounce=2, nrm=dnrm)
    d, pdf = d.cpu().numpy().astype(np.float64), pdf.cpu().numpy().astype(np.float64)
    assert np.allclose(np.linalg.norm(d, axis=0), 1, atol=1e-6)
    uv = orc.oct_encode_many(d)
    b = np.minimum((uv * 16).astype(np.int64), 15)
    frac = uv * 16 - np.floor(uv * 16)
    inner = ((frac > 1e-4) & (frac < 1 - 1e-4)).all(0)
    assert inner.mean() > 0.99
    bin_ = b[1] * 16 + b[0]
    want = prob[np.arange(len(bin_)), bin_] * 256 / FOUR_PI
    np.testing.assert_allclose(pdf[inner], want[inner], rtol=1e-5)
    st = w.learned_stats(g)
    assert st["fallbacks"] == 0 and math.isfinite(st["last_probe_kl"])


def test_learned_sample_chi_square(orc, w, torch_dev, box):
    """All vertices at one position: the sampled bins follow the network's
    distribution (chi-square over bins with expected count >= 5)."""
    cfg = orc.nn_cfg(**SMALL)
    n_par = orc.nn_num_params(cfg)
    g = small_model(w, torch_dev, box["rects"])
    params = nn_params.random_params(n_par, np.random.default_rng(9), scale=1.0)
    w.nn_set_params(g, params)
    n = 200_000
    pos = np.repeat(box["pos"][:, :1], n, axis=1)
    nrm = np.repeat(box["nrm"][:, :1], n, axis=1)
    dpos, dnrm = dev(torch_dev, pos), dev(torch_dev, nrm)
    p = w.nn_forward(g, dpos[:, :1].contiguous(), dnrm[:, :1].contiguous()).cpu().numpy()[0].astype(np.float64)
    opts = w.make_opts(N=16, mode=1, kl_bound=1e30, probe_stride=1024)
    d, _ = w.guide_sample(g, dpos, opts, seed=3, bounce=0, nrm=dnrm)
    uv = orc.oct_encode_many(d.cpu().numpy().astype(np.float64))
    b = np.minimum((uv * 16).astype(np.int64), 15)
    cnt = np.bincount(b[1] * 16 + b[0], minlength=256).astype(np.float64)
    exp = p * n
    big = exp >= 5
    chi2 = (((cnt - exp) ** 2 / exp)[big]).sum() + ((cnt[~big].sum() - exp[~big].sum()) ** 2 /
                                                    max(exp[~big].sum(), 1e-9) if (~big).any() else 0)
    dof = big.sum() + (1 if (~big).any() else 0) - 1
    from scipy.stats import chi2 as chi2d
    assert chi2d.sf(chi2, dof) > 1e-4, (chi2, dof)


# ------------------------------------------------- training and judge ----
@pytest.fixture(scope="module")
def trained(w, torch_dev, box):
    """Cornell box model trained on march pdfs of surface points."""
    rects, g = box["rects"], box["g"]
    pos, nrm, _ = synth.area_points(rects, 131072, 22)
    dpos, dnrm = dev(torch_dev, pos), dev(torch_dev, nrm)
    hpos_h, hnrm_h, _ = synth.area_points(rects, 4096, 23)      # held out
    hpos, hnrm = dev(torch_dev, hpos_h), dev(torch_dev, hnrm_h)
    target = box["o"].guide_pdf(hpos_h, 16) * FOUR_PI / 256     # the oracle's march distribution
    target /= target.sum(1, keepdims=True)
    w.guide_train(g, dpos, dnrm, steps=0, seed=1, n_max=64)
    kl_init = kl_to(w, g, hpos, hnrm, target)
    losses = [w.guide_train(g, dpos, dnrm, steps=100, batch=16384, n_max=64) for _ in range(4)]
    kl_trained = kl_to(w, g, hpos, hnrm, target)
    return dict(g=g, dpos=dpos, dnrm=dnrm, hpos=hpos, hnrm=hnrm, hpos_h=hpos_h, target=target,
                kl_init=kl_init, kl_trained=kl_trained, losses=losses)


def kl_to(w, g, hpos, hnrm, target):
    import oracle
    q = w.nn_forward(g, hpos, hnrm).cpu().numpy().astype(np.float64)
    return float(oracle.kl_rows(target, q).mean())


def test_training_learns_march_pdfs(trained):
    t = trained
    assert t["losses"][-1] < t["losses"][0]
    # held-out vertices: the trained network is far closer to the march than
    # the initial one. (On this scene every leaf-side carries an independent
    # LogNormal exitance, so the march pdf jumps whenever a vertex moves by a
    # leaf: the held-out KL has a floor that no smooth interpolant removes.)
    assert t["kl_trained"] < 0.4 * t["kl_init"], (t["kl_trained"], t["kl_init"])


def test_judge_kl_is_probe_mean(orc, w, torch_dev, trained):
    t, g = trained, trained["g"]
    hpos, hnrm = t["hpos"], t["hnrm"]
    stride = 16
    opts = w.make_opts(N=16, mode=1, kl_bound=1e30, probe_stride=stride)
    w.guide_sample(g, hpos, opts, seed=1, bounce=0, nrm=hnrm)
    kl = w.learned_stats(g)["last_probe_kl"]
    q = w.nn_forward(g, hpos, hnrm).cpu().numpy().astype(np.float64)
    want = float(orc.kl_rows(t["target"][::stride], q[::stride]).mean())
    assert abs(kl - want) <= 1e-3 * want + 1e-6, (kl, want)


@pytest.mark.parametrize("eps,blur", [(0.1, False), (0.01, True), (0.3, True)])
def test_judge_uses_the_fallback_field(orc, w, torch_dev, box, trained, eps, blur):
    """The judge's probes are marched with the caller's eps and blur, the
    field the fallback would sample: its KL equals the oracle's KL of the
    network against that field (Sec. 4 initial value and blur)."""
    t, g = trained, trained["g"]
    stride = 16
    opts = w.make_opts(N=16, eps=eps, mode=1, kl_bound=1e30, probe_stride=stride, blur=blur)
    w.guide_sample(g, t["hpos"], opts, seed=1, bounce=0, nrm=t["hnrm"])
    kl = w.learned_stats(g)["last_probe_kl"]
    q = w.nn_forward(g, t["hpos"], t["hnrm"]).cpu().numpy().astype(np.float64)[::stride]
    L = box["o"].field_aa(np.ascontiguousarray(t["hpos_h"][:, ::stride]), 16, blur=blur, eps=eps)
    target = L / L.sum(1, keepdims=True)
    want = float(orc.kl_rows(target, q).mean())
    assert abs(kl - want) <= 1e-3 * want + 1e-6, (kl, want)
    # and a bound the network misses makes the call return that field's march samples
    d0, p0 = w.guide_sample(g, t["hpos"], w.make_opts(N=16, eps=eps, blur=blur), seed=3, bounce=1)
    d1, p1 = w.guide_sample(g, t["hpos"], w.make_opts(N=16, eps=eps, mode=1, kl_bound=0.0, blur=blur),
                            seed=3, bounce=1, nrm=t["hnrm"])
    assert np.array_equal(p0.cpu().numpy().view(np.uint32), p1.cpu().numpy().view(np.uint32))
    assert np.array_equal(d0.cpu().numpy().view(np.uint32), d1.cpu().numpy().view(np.uint32))


def test_fallback_is_the_march_bit_for_bit(w, torch_dev, trained):
    g, hpos, hnrm = trained["g"], trained["hpos"], trained["hnrm"]
    before = w.learned_stats(g)["fallbacks"]
    d0, p0 = w.guide_sample(g, hpos, w.make_opts(N=16), seed=5, bounce=3)
    d1, p1 = w.guide_sample(g, hpos, w.make_opts(N=16, mode=1, kl_bound=0.0), seed=5, bounce=3, nrm=hnrm)
    assert w.learned_stats(g)["fallbacks"] == before + 1
    assert np.array_equal(d0.cpu().numpy().view(np.uint32), d1.cpu().numpy().view(np.uint32))
    assert np.array_equal(p0.cpu().numpy().view(np.uint32), p1.cpu().numpy().view(np.uint32))
    # within the bound: the network's samples (they differ from the march's)
    d2, p2 = w.guide_sample(g, hpos, w.make_opts(N=16, mode=1, kl_bound=1.0), seed=5, bounce=3, nrm=hnrm)
    assert w.learned_stats(g)["fallbacks"] == before + 1
    assert not np.array_equal(p0.cpu().numpy(), p2.cpu().numpy())


def test_learned_errors(w, torch_dev, box):
    g = w.svo_build(box["rects"], 6)
    pos, nrm = dev(torch_dev, box["pos"]), dev(torch_dev, box["nrm"])
    with pytest.raises(w.WfpgError) as e:
        w.guide_sample(g, pos, w.make_opts(N=16, mode=1), seed=0, bounce=0, nrm=nrm)
    assert e.value.status == -4
    with pytest.raises(w.WfpgError):
        w.nn_get_params(g)
    with pytest.raises(w.WfpgError) as e:
        w.guide_train(g, pos, nrm, steps=1, log2_table=30)
    assert e.value.status == -1
    w.guide_train(g, pos, nrm, steps=0)
    with pytest.raises(w.WfpgError) as e:      # the learned field is 16 x 16
        w.guide_sample(g, pos, w.make_opts(N=8, mode=1), seed=0, bounce=0, nrm=nrm)
    assert e.value.status == -1
    with pytest.raises(w.WfpgError) as e:      # normals are inputs of the network
        w.guide_sample(g, pos, w.make_opts(N=16, mode=1), seed=0, bounce=0)
    assert e.value.status == -1


def test_uniform_enclosure_target_is_learned(orc, w, torch_dev):
    """Closed room with the same exitance on both sides of every leaf: every
    bin of an interior point hits, so the march pdf is uniform (a closed
    form); the trained network reaches KL < 1e-4 against it."""
    import oracle
    rects = synth.room(n_boxes=8)
    D = 6
    o = oracle.SVO(rects, D)
    xyz, _ = o.leaf_info()
    nrm = o.normals(D).astype(np.float32)
    L = xyz.shape[0]
    p = ((xyz.astype(np.float64) + 0.5) / (1 << D)).T.astype(np.float32)
    pos = np.ascontiguousarray(np.concatenate([p, p], 1))
    wo = np.ascontiguousarray(np.concatenate([nrm.T, -nrm.T], 1))
    rgb = np.ones((3, 2 * L), np.float32)
    g = w.svo_build(rects, D)
    w.svo_accumulate(g, dev(torch_dev, pos), dev(torch_dev, wo), dev(torch_dev, rgb))
    # interior points (a point on a wall sees the outside through half its
    # directions); the normal input is an arbitrary unit vector
    rng = np.random.default_rng(31)
    vp = rng.uniform(0.02, 0.98, (3, 65536)).astype(np.float32)
    vn = rng.normal(size=(3, 65536))
    vn = (vn / np.linalg.norm(vn, axis=0)).astype(np.float32)
    dpos, dnrm = dev(torch_dev, vp), dev(torch_dev, vn)
    t = w.guide_pdf(g, dpos[:, :256].contiguous(), w.make_opts(N=16)).cpu().numpy()
    np.testing.assert_allclose(t, 1 / FOUR_PI, rtol=1e-5)
    w.guide_train(g, dpos, dnrm, steps=300, batch=8192)
    q = w.nn_forward(g, dpos, dnrm).cpu().numpy().astype(np.float64)
    kl = orc.kl_rows(np.full_like(q, 1 / 256), q)
    assert kl.mean() < 1e-4, kl.mean()


def test_forward_full_size_configuration(orc, w, torch_dev):
    """The configuration the bench trains (16 levels x 2^19 entries, N_min 16,
    N_max 2^10 on a depth-10 SVO): resolutions, dense/hashed levels and the
    forward pass agree with the oracle."""
    rects = synth.room(n_boxes=8)
    g = w.svo_build(rects, 10)
    pos, nrm, _ = synth.area_points(rects, 200, 41)
    w.guide_train(g, dev(torch_dev, pos), dev(torch_dev, nrm), steps=0)
    cfg = orc.nn_cfg(log2_table=19, n_min=16, n_max=1024)
    n_par = orc.nn_num_params(cfg)
    assert w.nn_param_count(g) == n_par
    params = nn_params.random_params(n_par, np.random.default_rng(12))
    w.nn_set_params(g, params)
    prob = w.nn_forward(g, dev(torch_dev, pos), dev(torch_dev, nrm)).cpu().numpy().astype(np.float64)
    p1, _ = orc.nn_forward(params, cfg, pos, nrm, mode=1)
    kl = orc.kl_rows(p1, prob)
    assert kl.max() < 1e-5, kl.max()
    pe, _ = orc.nn_parity_bounds(params, cfg, pos, nrm)
    rel = np.abs(prob - p1) / p1
    bars.record("nn forward full size rel / bound", (rel / pe).max(), 1.0)
    assert (rel <= pe).all(), (rel / pe).max()


def test_learned_faster_than_march_within_bound(orc, w, torch_dev):
    """What the trained network gains over the march: on the frame-scale room
    with the field blurred and eps = 1 (Sec. 4: the field's initial value and
    its Gaussian blur), a network trained on that field by the library's own
    kernels passes the judge (probe KL <= 0.05, no fallback), its mean
    per-vertex KL against the oracle's field is within 0.05 on strided
    camera-queue vertices, and mode 1 returns the 2,073,600 samples faster
    than the march."""
    torch, device = torch_dev
    import oracle
    room = synth.room()
    sp = synth.room_splats(room, 2_000_000, 13)
    o = oracle.SVO(room, 10)
    o.accumulate(*sp)
    o.propagate()
    g = w.svo_build(room, 10)
    w.svo_accumulate(g, *[dev(torch_dev, a) for a in sp])
    cam, cn, _ = synth.camera_queue(room)
    frames = [synth.camera_queue(room, jitter_seed=200 + f)[:2] for f in range(2)]
    tp = np.concatenate([f[0] for f in frames], 1)
    tn = np.concatenate([f[1] for f in frames], 1)
    perm = np.random.default_rng(3).permutation(tp.shape[1])
    w.guide_train(g, dev(torch_dev, tp[:, perm]), dev(torch_dev, tn[:, perm]), steps=500, batch=65536,
                  target_eps=1.0, target_blur=1)
    pos, nrm = dev(torch_dev, cam), dev(torch_dev, cn)
    idx = np.arange(0, cam.shape[1], cam.shape[1] // 2048)
    L = o.field_aa(np.ascontiguousarray(cam[:, idx]), 16, blur=True, eps=1.0)
    t = L / L.sum(1, keepdims=True)
    q = w.nn_forward(g, dev(torch_dev, cam[:, idx]), dev(torch_dev, cn[:, idx])).cpu().numpy().astype(np.float64)
    kl = orc.kl_rows(t, q)
    bars.record("learned eps=1 blur KL mean (oracle field)", kl.mean(), 0.05)
    assert kl.mean() <= 0.05, kl.mean()
    o1 = w.make_opts(N=16, eps=1.0, blur=True, mode=1, kl_bound=0.05, probe_stride=256)
    o0 = w.make_opts(N=16, eps=1.0, blur=True)
    n = cam.shape[1]
    d, p = torch.empty((3, n), device=device), torch.empty((n,), device=device)

    def ms_of(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return sorted(ts)[2]
    fb = w.learned_stats(g)["fallbacks"]
    m1 = ms_of(lambda: w.guide_sample(g, pos, o1, seed=4, bounce=0, nrm=nrm, dir_out=d, pdf_out=p))
    st = w.learned_stats(g)
    assert st["fallbacks"] == fb and st["last_probe_kl"] <= 0.05, st
    assert torch.isfinite(p).all() and (p > 0).all()
    m0 = ms_of(lambda: w.guide_sample(g, pos, o0, seed=4, bounce=0, dir_out=d, pdf_out=p))
    bars.record("learned mode-1 speedup over the march (eps=1, blur)", m0 / m1)
    assert m1 < m0, (m1, m0)
