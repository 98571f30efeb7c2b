"""Pins of the oracle's exitance extraction (Eq. 5): the splats a wavefront's
path memory yields when its paths reach emitters.

Checked against what Eq. 5 fixes: the radiance at depth k is the emitted
radiance times the product of the path's throughput factors after k (built
here from independent FP64 factors), exactly L_e at the emitter's own depth;
every depth 1..n of a path with an emitter yields one splat, paths without
one none; the outgoing direction points from p_k back to p_{k-1} (the eye for
k = 1); and the splats land in the SVO as plain splats do.
"""
import numpy as np
import pytest

import oracle
import synth


def factor_paths(P, d, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.2, 0.9, (d, 3, P))
    T = np.cumprod(f, axis=0).astype(np.float32)          # T_k = prod_{j<=k} f_j
    return f, T


def test_radiance_is_the_product_of_later_factors():
    P, d = 500, 6
    rects = synth.cornell_box()
    pos, _, eye, hit, Le = synth.path_wavefront(rects, P, d, seed=4, hit_prob=1.0)
    f, T = factor_paths(P, d, 9)
    sp, sw, sr = oracle.path_splats(pos, T, eye, hit, Le)
    assert sp.shape[1] == hit.sum()
    m = 0
    want = np.zeros((3, sp.shape[1]))
    for k in range(1, d + 1):
        for i in range(P):
            if hit[i] >= k:
                want[:, m] = np.prod(f[k:hit[i], :, i], axis=0) * Le[:, i]
                m += 1
    np.testing.assert_allclose(sr, want, rtol=2e-6 * d)


def test_emitter_depth_gets_le_and_directions_point_back():
    P, d = 300, 5
    rects = synth.cornell_box()
    pos, T, eye, hit, Le = synth.path_wavefront(rects, P, d, seed=5)
    sp, sw, sr = oracle.path_splats(pos, T, eye, hit, Le)
    valid = (hit >= 1)
    assert sp.shape[1] == hit[valid].sum()
    m = 0
    for k in range(1, d + 1):
        for i in range(P):
            if valid[i] and hit[i] >= k:
                assert np.array_equal(sp[:, m], pos[k - 1, :, i])
                prev = eye[:, i] if k == 1 else pos[k - 2, :, i]
                assert np.array_equal(sw[:, m], (prev - pos[k - 1, :, i]).astype(np.float32))
                if k == hit[i]:
                    assert np.array_equal(sr[:, m], Le[:, i])
                m += 1


def test_no_emitter_no_splats_and_unit_throughput():
    P, d = 64, 4
    rects = synth.cornell_box()
    pos, T, eye, hit, Le = synth.path_wavefront(rects, P, d, seed=6)
    sp, _, _ = oracle.path_splats(pos, T, eye, np.full(P, -1, np.int32), Le)
    assert sp.shape[1] == 0
    sp, _, _ = oracle.path_splats(pos, T, eye, np.zeros(P, np.int32), Le)
    assert sp.shape[1] == 0
    ones = np.ones_like(T)
    full = np.full(P, d, np.int32)
    _, _, sr = oracle.path_splats(pos, ones, eye, full, Le)
    np.testing.assert_array_equal(sr, np.tile(Le, (1, d)))
    # a zero throughput channel gives a zero ratio, not NaN
    Tz = T.copy()
    Tz[0, 1, :] = 0.0
    _, _, sr = oracle.path_splats(pos, Tz, eye, full, Le)
    assert np.isfinite(sr).all() and (sr[1, :P] == 0).all()


def test_splats_accumulate_as_plain_splats(orc):
    rects = synth.cornell_box()
    o = orc.SVO(rects, 6)
    P, d = 4000, 8
    pos, T, eye, hit, Le = synth.path_wavefront(rects, P, d, seed=7)
    sp, sw, sr = oracle.path_splats(pos, T, eye, hit, Le)
    assert o.accumulate(sp, sw, sr) == 0          # surface points sit in occupied leaves
    _, s64, cnt = o.leaf_accum()
    assert cnt.sum() == sp.shape[1]
    f = np.float32
    y = (f(0.2126) * sr[0] + f(0.7152) * sr[1]) + f(0.0722) * sr[2]   # the splat luminance, FP32
    assert s64.sum() == pytest.approx(y.astype(np.float64).sum(), rel=1e-12)
