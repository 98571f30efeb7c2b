"""Pins of the learned-model oracle: central finite differences of the FP64
network, exact reproduction of linear fields by the trilinear hash
interpolation on dense levels, closed forms of the softmax cross-entropy and
of KL, and the BF16-faithful mode staying close to FP64."""
import math

import numpy as np
import pytest

import nn_params
import synth

SMALL = dict(log2_table=12, n_min=4, n_max=64)


def layout(o, cfg):
    return nn_params.layout(o.nn_num_params(cfg))


def random_params(o, cfg, rng, scale=0.3, table_scale=0.5):
    return nn_params.random_params(o.nn_num_params(cfg), rng, scale, table_scale)


def test_resolutions_and_sizes(orc):
    cfg = orc.nn_cfg()
    r = orc.nn_resolutions(cfg)
    assert r[0] == 16 and r[-1] in (1023, 1024) and (np.diff(r) > 0).all()
    b = math.exp((math.log(1024) - math.log(16)) / 15)
    assert abs(r[7] - 16 * b ** 7) < 1.0
    assert orc.nn_mlp_params() == 35 * 64 + 64 + 3 * (64 * 64 + 64) + 256 * 64 + 256 == 31424
    assert orc.nn_num_params(cfg) == 31424 + 16 * (1 << 19) * 2


def test_finite_differences_fp64(orc):
    cfg = orc.nn_cfg(**SMALL)
    rng = np.random.default_rng(0)
    params = random_params(orc, cfg, rng).astype(np.float64)
    room = synth.room(n_boxes=4)
    pos, nrm, _ = synth.area_points(room, 3, 1)
    t = rng.random((3, 256)) ** 4
    t /= t.sum(1, keepdims=True)
    loss, g = orc.nn_grad(params.astype(np.float32), cfg, pos, nrm, t, mode=0)
    lay = layout(orc, cfg)
    # probe: weights and biases of every layer, and table entries actually touched
    probes = []
    for name in ["W0", "b0", "W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]:
        a, m = lay[name]
        probes += list(a + rng.choice(m, 4, replace=False))
    a, m = lay["table"]
    touched = np.nonzero(g[a:a + m])[0]
    probes += list(a + rng.choice(touched, 8, replace=False))
    base = params.astype(np.float32)
    for idx in probes:
        h = max(1e-3 * abs(float(base[idx])), 1e-3)
        # parameters are FP32; use exactly representable perturbations
        up, dn = base.copy(), base.copy()
        up[idx] = np.float32(base[idx] + h)
        dn[idx] = np.float32(base[idx] - h)
        hh = (float(up[idx]) - float(dn[idx])) / 2
        lu, _ = orc.nn_grad(up, cfg, pos, nrm, t, mode=0)
        ld, _ = orc.nn_grad(dn, cfg, pos, nrm, t, mode=0)
        fd = (lu - ld) / (2 * hh)
        assert abs(fd - g[idx]) <= 1e-5 * max(1.0, abs(fd)) + 5e-7, (idx, fd, g[idx])


def test_uniform_softmax_closed_form(orc):
    cfg = orc.nn_cfg(**SMALL)
    rng = np.random.default_rng(1)
    params = random_params(orc, cfg, rng)
    lay = layout(orc, cfg)
    for name in ("W4", "b4"):
        a, m = lay[name]
        params[a:a + m] = 0
    room = synth.room(n_boxes=4)
    pos, nrm, _ = synth.area_points(room, 5, 2)
    prob, logit = orc.nn_forward(params, cfg, pos, nrm, mode=0)
    np.testing.assert_allclose(prob, 1 / 256, rtol=1e-14)
    t = np.full((5, 256), 1 / 256)
    loss, g = orc.nn_grad(params, cfg, pos, nrm, t, mode=0)
    assert abs(loss - math.log(256)) < 1e-12
    a, m = lay["b4"]
    assert np.abs(g[a:a + m]).max() < 1e-15
    # a one-hot target: dL/db4 = p - onehot, averaged
    t1 = np.zeros((5, 256))
    t1[:, 7] = 1
    loss1, g1 = orc.nn_grad(params, cfg, pos, nrm, t1, mode=0)
    assert abs(loss1 - math.log(256)) < 1e-12
    want = np.full(256, 1 / 256)
    want[7] -= 1
    np.testing.assert_allclose(g1[a:a + m], want, atol=1e-15)


def test_trilinear_reproduces_linear_fields(orc):
    """On dense levels, a table holding a linear function of the corner
    coordinates interpolates to the same linear function of p * R."""
    cfg = orc.nn_cfg(**SMALL)
    res = orc.nn_resolutions(cfg)
    T = 1 << SMALL["log2_table"]
    lay = layout(orc, cfg)
    params = np.zeros(orc.nn_num_params(cfg), np.float32)
    a, _ = lay["table"]
    coef = np.array([[0.25, -0.5, 0.125, 1.0], [0.5, 0.25, -0.25, -2.0]])   # per feature
    dense = []
    for l, R in enumerate(res):
        side = R + 1
        if side ** 3 > T:
            continue
        dense.append(l)
        z, y, x = np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij")
        idx = (x + side * (y + side * z)).ravel()
        for f in range(2):
            vals = coef[f, 0] * x.ravel() + coef[f, 1] * y.ravel() + coef[f, 2] * z.ravel() + coef[f, 3]
            params[a + (l * T + idx) * 2 + f] = vals
    assert len(dense) >= 2
    rng = np.random.default_rng(4)
    pos = rng.random((3, 50)).astype(np.float32)
    nrm = np.zeros((3, 50), np.float32)
    # read the encoded features through the first layer: W0 = identity on them
    a0, _ = lay["W0"]
    for l in dense:
        W = np.zeros((64, 35), np.float32)
        W[0, 2 * l] = 1.0
        W[1, 2 * l + 1] = 1.0
        params[a0:a0 + 64 * 35] = W.ravel()
        # identity through the hidden layers on units 0, 1 (values kept positive by an offset)
        p2 = params.copy()
        off = {"b0": 100.0}
        b0a, _ = lay["b0"]
        p2[b0a:b0a + 64] = 0
        p2[b0a] = p2[b0a + 1] = 100.0
        for k in (1, 2, 3):
            wa, _ = lay["W%d" % k]
            Wk = np.zeros((64, 64), np.float32)
            Wk[0, 0] = Wk[1, 1] = 1
            p2[wa:wa + 64 * 64] = Wk.ravel()
        w4a, _ = lay["W4"]
        W4 = np.zeros((256, 64), np.float32)
        W4[0, 0] = W4[1, 1] = 1
        p2[w4a:w4a + 256 * 64] = W4.ravel()
        _, logit = orc.nn_forward(p2, cfg, pos, nrm, mode=0)
        xs = pos.astype(np.float32) * np.float32(res[l])
        for f in range(2):
            want = (coef[f, 0] * xs[0].astype(np.float64) + coef[f, 1] * xs[1] + coef[f, 2] * xs[2] +
                    coef[f, 3] + 100.0)
            # fractions and 1 - fraction are FP32 (the cell choice is taken in FP32),
            # so the weights carry FP32 rounding: |error| <= ~4 * 2^-24 * sum |values|
            np.testing.assert_allclose(logit[:, f], want, rtol=0, atol=4e-6)


def test_kl_closed_forms(orc):
    p = np.array([[0.5, 0.5] + [0.0] * 254])
    q = np.array([[0.25, 0.75] + [0.0] * 254])
    q[0, 2:] = 0
    kl = orc.kl_rows(p, q)[0]
    want = 0.5 * math.log(0.5 / 0.25) + 0.5 * math.log(0.5 / 0.75)
    assert abs(kl - want) < 1e-15
    r = np.random.default_rng(0).random((4, 256))
    r /= r.sum(1, keepdims=True)
    assert np.abs(orc.kl_rows(r, r)).max() < 1e-15


def test_bf16_faithful_close_to_fp64(orc):
    cfg = orc.nn_cfg(**SMALL)
    rng = np.random.default_rng(5)
    params = random_params(orc, cfg, rng)
    room = synth.room(n_boxes=4)
    pos, nrm, _ = synth.area_points(room, 16, 3)
    p0, _ = orc.nn_forward(params, cfg, pos, nrm, mode=0)
    p1, _ = orc.nn_forward(params, cfg, pos, nrm, mode=1)
    kl = orc.kl_rows(p0, p1)
    assert kl.max() < 1e-3
    t = rng.random((16, 256))
    t /= t.sum(1, keepdims=True)
    _, g0 = orc.nn_grad(params, cfg, pos, nrm, t, mode=0)
    _, g1 = orc.nn_grad(params, cfg, pos, nrm, t, mode=1)
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 0.05
