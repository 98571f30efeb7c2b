"""Pins of the network oracle's parity bounds (orc_nn_parity_bounds): an FP32
implementation of the same network, written here in numpy with every sum
taken in a random order and BF16 roundings where the kernels round, lands
within the bounds the oracle states around its BF16-faithful mode, for every
probability and every gradient element; the bounds are not vacuous; and
the BF16 interval of a pre-activation on closed-form cases (on a rounding
boundary, near it, exactly representable, zero)."""
import numpy as np

import nn_params
import synth

SMALL = dict(log2_table=12, n_min=4, n_max=64)
FIN = nn_params.FIN
FOUT = nn_params.FOUT


def bf16(a):
    """Round FP32 values to BF16 (nearest, ties to even); returns float32."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32)


def fsum(terms, axis, rng):
    """FP32 sequential sum along `axis` in a random order of the terms."""
    t = np.take(np.asarray(terms, np.float32), rng.permutation(terms.shape[axis]), axis=axis)
    return np.take(np.cumsum(t, axis=axis, dtype=np.float32), -1, axis=axis)


def unpack(params):
    lay = nn_params.layout(params.size)
    W, B = [], []
    for k in range(5):
        a, m = lay["W%d" % k]
        W.append(params[a:a + m].reshape(FOUT[k], FIN[k]))
        a, m = lay["b%d" % k]
        B.append(params[a:a + m])
    return W, B, lay


def emulate(orc, params, cfg, pos, nrm, t32, rng):
    """FP32 forward and backward with BF16 roundings where the kernels round,
    every sum in a random order: (probabilities, gradient vector)."""
    W, B, lay = unpack(params)
    Wb = [bf16(w) for w in W]
    n = pos.shape[1]
    x = orc.nn_inputs(params, cfg, pos, nrm, mode=1).astype(np.float32)   # BF16 values, exact in FP32
    acts = [x]
    h = x
    for k in range(4):
        terms = np.concatenate([Wb[k][None, :, :] * h[:, None, :],
                                np.broadcast_to(B[k][None, :, None], (n, FOUT[k], 1))], 2)
        a = fsum(terms, 2, rng)
        h = bf16(np.maximum(a, 0))
        acts.append(h)
    terms = np.concatenate([Wb[4][None, :, :] * h[:, None, :], np.broadcast_to(B[4][None, :, None], (n, 256, 1))], 2)
    z = fsum(terms, 2, rng)
    e = np.exp((z - z.max(1, keepdims=True)).astype(np.float32)).astype(np.float32)
    p = (e / fsum(e, 1, rng)[:, None]).astype(np.float32)
    if t32 is None:
        return p, None
    grad = np.zeros(params.size, np.float64)
    inv_b = np.float32(1.0 / n)
    tt = (t32 / fsum(t32, 1, rng)[:, None]).astype(np.float32)
    g = ((p - tt) * inv_b).astype(np.float32)
    dzr = bf16(g)
    a_, m_ = lay["b4"]
    grad[a_:a_ + m_] = fsum(g, 0, rng)
    a_, m_ = lay["W4"]
    grad[a_:a_ + m_] = fsum(dzr[:, :, None] * acts[4][:, None, :], 0, rng).reshape(-1)
    dh = fsum(Wb[4][None, :, :] * dzr[:, :, None], 1, rng)            # (n, 64)
    for k in range(3, -1, -1):
        da = np.where(acts[k + 1] > 0, dh, 0).astype(np.float32)
        dar = bf16(da)
        a_, m_ = lay["b%d" % k]
        grad[a_:a_ + m_] = fsum(da, 0, rng)
        a_, m_ = lay["W%d" % k]
        grad[a_:a_ + m_] = fsum(dar[:, :, None] * acts[k][:, None, :], 0, rng).reshape(-1)
        dh = fsum(Wb[k][None, :, :] * dar[:, :, None], 1, rng)        # (n, FIN[k])
    # table: FP32 products of the corner weight and the input gradient,
    # accumulated in FP32 in a random order of all (row, corner) terms
    a_, m_ = lay["table"]
    T = 1 << cfg.log2_table
    contrib = {}
    for i in range(n):
        idx, wgt = orc.nn_encode_info(cfg, pos[:, i])
        for l in range(16):
            for q in range(8):
                for f in range(2):
                    key = (l * T + int(idx[l, q])) * 2 + f
                    contrib.setdefault(key, []).append(np.float32(np.float32(wgt[l, q]) * dh[i, 2 * l + f]))
    for key, vals in contrib.items():
        v = np.array(vals, np.float32)[rng.permutation(len(vals))]
        grad[a_ + key] = np.cumsum(v, dtype=np.float32)[-1]
    return p, grad


def setup(orc, seed, n):
    cfg = orc.nn_cfg(**SMALL)
    rng = np.random.default_rng(seed)
    params = nn_params.random_params(orc.nn_num_params(cfg), rng)
    room = synth.room(n_boxes=6)
    pos, nrm, _ = synth.area_points(room, n, seed + 100)
    t32 = (rng.random((n, 256)) ** 4).astype(np.float32)
    t32 /= t32.sum(1, keepdims=True)
    return cfg, params, pos, nrm, t32


def test_forward_within_bounds(orc):
    cfg, params, pos, nrm, _ = setup(orc, 1, 160)
    pe, _ = orc.nn_parity_bounds(params, cfg, pos, nrm)
    p1, _ = orc.nn_forward(params, cfg, pos, nrm, mode=1)
    assert np.median(pe) < 1e-3, np.median(pe)            # not vacuous
    for s in range(4):
        p, _ = emulate(orc, params, cfg, pos, nrm, None, np.random.default_rng(10 + s))
        rel = np.abs(p.astype(np.float64) - p1) / p1
        assert (rel <= pe).all(), (rel / pe).max()


def test_gradient_within_bounds(orc):
    cfg, params, pos, nrm, t32 = setup(orc, 2, 64)
    t = t32.astype(np.float64)
    t /= t.sum(1, keepdims=True)
    B = 64   # a power of two: the batch scale 1/B is exact in FP32
    _, gr = orc.nn_parity_bounds(params, cfg, pos, nrm, target=t, inv_b=1.0 / B)
    _, g1 = orc.nn_grad(params, cfg, pos, nrm, t, mode=1)
    lay = nn_params.layout(params.size)
    # tight near the output; worst-case flips compound towards the input
    for name, lim in (("b4", 0.02), ("W4", 0.1), ("W3", 0.3), ("b3", 0.3)):
        a, m = lay[name]
        rel = gr[a:a + m] / np.maximum(np.abs(g1[a:a + m]), 1e-300)
        assert np.median(rel) < lim, (name, np.median(rel))
    for s in range(2):
        _, g = emulate(orc, params, cfg, pos, nrm, t32, np.random.default_rng(20 + s))
        d = np.abs(g - g1)
        bad = d > gr * (1 + 1e-9) + 1e-300
        assert not bad.any(), (np.nonzero(bad)[0][:10], (d / np.maximum(gr, 1e-300)).max())


def test_interval_closed_forms(orc):
    """Zero weights: every pre-activation of layer 0 is its FP32 bias, within
    2 * 65 * u * |b|. A bias on a BF16 rounding boundary (1 + 2^-8) or within
    the bound of it may round to either neighbour (radius 2^-7 around 1 or
    1 + 2^-7, which moves the logits only through W4 = 0: no effect on p);
    exactly representable ones, one outside the bound and 0 have radius 0.
    The relative bound of the uniform distribution is then the softmax's own
    (256 bins of equal logits)."""
    cfg = orc.nn_cfg(**SMALL)
    n_par = orc.nn_num_params(cfg)
    lay = nn_params.layout(n_par)
    pos, nrm, _ = synth.area_points(synth.room(n_boxes=2), 4, 3)
    u = 2.0 ** -24
    params = np.zeros(n_par, np.float32)
    a, m = lay["b0"]
    for b in (1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, 0.0):
        params[a:a + m] = np.float32(b)
        pe, _ = orc.nn_parity_bounds(params, cfg, pos, nrm)
        np.testing.assert_allclose(pe, np.expm1((4 + 512 + 2) * u), rtol=1e-12)
    # with the later layers' weights nonzero a layer-0 flip reaches the
    # logits: the tie bias gives a larger bound than the representable one
    rng = np.random.default_rng(0)
    for name in ("W1", "W2", "W3", "W4"):
        a2, m2 = lay[name]
        params[a2:a2 + m2] = rng.normal(0, 0.1, m2).astype(np.float32)
    params[a:a + m] = np.float32(1.0)
    pe_exact, _ = orc.nn_parity_bounds(params, cfg, pos, nrm)
    params[a:a + m] = np.float32(1.0 + 2.0 ** -8)
    pe_tie, _ = orc.nn_parity_bounds(params, cfg, pos, nrm)
    assert (pe_tie >= pe_exact).all() and pe_tie.mean() > 2 * pe_exact.mean()
