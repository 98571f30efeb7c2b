"""Pins of the oracle's field antialiasing (Sec. 4): directional jitter of the
cone directions and the Gaussian blur of the field.

Jitter: every jittered direction is a unit vector inside its own bin, at the
offset the Philox stream (pinned by its known-answer test) gives, and the
offsets are uniform over the bin. Blur: a constant field is a fixed point;
the operator is symmetric with unit row sums (so it keeps the field's total);
an interior delta spreads as the binomial stencil; and every neighbour the
edge folding picks is a geometric neighbour on the sphere (an error in the
folding, e.g. wrapping around like a torus, puts it far away).
"""
import numpy as np
import pytest

import oracle
import synth


def offsets(N, key):
    o = np.array([oracle.philox([b, 0, 0, 3], [key, 0]) for b in range(N * N)], np.uint64)
    return (o[:, 0] >> 8) * 2.0 ** -24, (o[:, 1] >> 8) * 2.0 ** -24


@pytest.mark.parametrize("N,key", [(8, 1), (16, 77), (32, 123456789), (128, 5)])
def test_jitter_directions_in_bin_at_philox_offset(N, key):
    t = oracle.jitter_table(N, key).astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(t, axis=1), 1.0, atol=2e-7)
    uv = oracle.oct_encode_many(np.ascontiguousarray(t.T)) * N
    b = np.arange(N * N)
    ju, jv = offsets(N, key)
    # the encoded FP32 direction sits at (u + j_u, v + j_v) up to FP32 rounding
    assert np.abs(uv[0] - (b % N + ju)).max() < 2e-4 * N
    assert np.abs(uv[1] - (b // N + jv)).max() < 2e-4 * N
    inner = (np.minimum(ju, 1 - ju) > 1e-3 * N) & (np.minimum(jv, 1 - jv) > 1e-3 * N)
    assert (np.floor(uv[0][inner]) == (b % N)[inner]).all() and (np.floor(uv[1][inner]) == (b // N)[inner]).all()
    # a different key moves every cone
    t2 = oracle.jitter_table(N, key + 1).astype(np.float64)
    assert (np.abs(t2 - t).max(1) > 0).all()


def test_jitter_offsets_uniform():
    from scipy.stats import kstest
    ju, jv = offsets(32, 99)
    assert kstest(ju, "uniform").pvalue > 1e-3 and kstest(jv, "uniform").pvalue > 1e-3


def blur_matrix(N):
    eye = np.eye(N * N)
    return oracle.blur(eye, N)                       # row k = blur of delta at k


@pytest.mark.parametrize("N", [8, 16])
def test_blur_operator_properties(N):
    B = blur_matrix(N)
    np.testing.assert_allclose(B, B.T, atol=1e-15)
    np.testing.assert_allclose(B.sum(1), 1.0, atol=1e-14)
    np.testing.assert_allclose(oracle.blur(np.full(N * N, 3.5), N), 3.5, rtol=1e-15)
    # interior delta: the binomial stencil
    u, v = N // 2, N // 2 - 1
    d = np.zeros((N, N))
    d[v, u] = 1.0
    out = oracle.blur(d.reshape(-1), N).reshape(N, N)
    st = np.outer([0.25, 0.5, 0.25], [0.25, 0.5, 0.25])
    np.testing.assert_allclose(out[v - 1:v + 2, u - 1:u + 2], st, atol=1e-15)
    assert out.sum() == pytest.approx(1.0) and np.count_nonzero(out) == 9


@pytest.mark.parametrize("N", [8, 16, 32])
def test_blur_neighbours_are_adjacent_on_the_sphere(N):
    """Each bin's 8 folded neighbours lie within 3 bin widths (angle) of it
    (the worst are diagonal neighbours of the elongated bins along the edge,
    about 2.3); a torus wrap at the square's edges would put some near the
    antipode, tens of widths away."""
    B = blur_matrix(N)
    c = oracle.dir_table(N).reshape(N * N, 3).astype(np.float64)
    width = np.sqrt(4 * np.pi / (N * N))
    worst = 0.0
    for k in range(N * N):
        nb = np.nonzero(B[k])[0]
        ang = np.arccos(np.clip(c[nb] @ c[k], -1, 1))
        worst = max(worst, ang.max() / width)
    assert worst < 3.0, worst


def test_blurred_field_guides_and_sums_like_the_field(orc):
    rects = synth.cornell_box()
    o = orc.SVO(rects, 6)
    xyz, em = o.leaf_info()
    o.accumulate(*synth.leaf_splats(xyz, o.normals(6), em, 6, seed=2))
    o.propagate()
    pos, _, _ = synth.area_points(rects, 200, 4)
    N = 16
    L = o.field_aa(pos, N)
    np.testing.assert_array_equal(L, o.field(pos, N)[0])            # no options: the plain field
    Lb = o.field_aa(pos, N, blur=True)
    np.testing.assert_allclose(Lb, oracle.blur(L, N), rtol=1e-15)
    np.testing.assert_allclose(Lb.sum(1), L.sum(1), rtol=1e-13)
    eps = float(np.float32(0.01))
    assert (Lb >= eps * (1 - 1e-12)).all()                          # stays above eps
    Lj = o.field_aa(pos, N, jitter_key=3)
    assert (Lj != L).any() and (Lj >= eps).all()
    # sampling the blurred field: the sampled bin's pdf is its blurred share
    r = oracle.sample_fields(Lb, N, 9, 1)
    b = r["bin"][:, 1] * N + r["bin"][:, 0]
    want = Lb / Lb.sum(1, keepdims=True) * (N * N) / (4 * np.pi)
    np.testing.assert_allclose(r["pdf"], want[np.arange(len(b)), b], rtol=1e-12)
