"""Pins of the oracle's product path guiding (Sec. 3.6): the two-level sampler
(8 x 8 upper level of summed field cells times the BSDF table, then the fine
bin inside the chosen cell) checked against what it must reach:

* the direct definition: the pdf of a bin is the normalized product of the
  fine field with the BSDF table held constant over each 8 x 8 cell;
* a closed form: a uniform field with a Lambertian normal +z gives cell
  probabilities z_C / 15, z_C = 1 - (|a| + |b|)^2 at the cell centre of the
  equal-area map (the 24 cells whose centre lies inside the upper diamond);
* special cases: a constant table, a zero or non-finite normal, N = 8;
* a chi-square of many samples of one field against the direct definition;
* normalization of the pdf over all bins, and sample/pdf consistency.
"""
import numpy as np
import pytest

import oracle
import synth


def f32_cos_table(nrm):
    """Lambertian table max(0, n . d_C) in FP32, (x x' + y y') + z z'."""
    d = oracle.dir_table(8).reshape(64, 3).astype(np.float32)
    n = np.asarray(nrm, np.float32)
    px = n[0][:, None] * d[None, :, 0]
    py = n[1][:, None] * d[None, :, 1]
    pz = n[2][:, None] * d[None, :, 2]
    x = (px + py) + pz
    return np.where(x > 0, x, np.float32(0)).astype(np.float64)


def direct_pdf(L, N, f):
    """pdf of every fine bin: L_b f_C(b) / sum(L f) * N^2 / (4 pi)."""
    s = N // 8
    fu = np.kron(f.reshape(-1, 8, 8), np.ones((1, s, s))).reshape(f.shape[0], N * N)
    prod = L * fu
    return prod / prod.sum(1, keepdims=True) * (N * N) / (4 * np.pi)


def rand_fields(n, N, seed):
    rng = np.random.default_rng(seed)
    # heavy-tailed positive values, like exitance + eps
    return rng.lognormal(0.0, 1.5, (n, N * N)) + 0.01


@pytest.mark.parametrize("N", [8, 16, 32, 64, 128])
def test_pdf_is_normalized_product_of_field_and_table(N):
    n = 400
    L = rand_fields(n, N, N)
    rng = np.random.default_rng(N + 1)
    nrm = rng.normal(size=(3, n)).astype(np.float32)
    r = oracle.product_sample_fields(L, N, 7, 3, nrm=nrm)
    want = direct_pdf(L, N, f32_cos_table(nrm))
    b = r["bin"][:, 1] * N + r["bin"][:, 0]
    np.testing.assert_allclose(r["pdf"], want[np.arange(n), b], rtol=1e-12)
    assert (want[np.arange(n), b] > 0).all()            # never a cell the table excludes
    # an arbitrary (non-symmetric) table: catches transposed cells
    tab = rng.uniform(0, 1, (n, 64)).astype(np.float32)
    tab[:, rng.integers(0, 64, 20)] = 0.0
    r = oracle.product_sample_fields(L, N, 7, 3, bsdf=tab)
    want = direct_pdf(L, N, tab.astype(np.float64))
    b = r["bin"][:, 1] * N + r["bin"][:, 0]
    np.testing.assert_allclose(r["pdf"], want[np.arange(n), b], rtol=1e-12)
    # the direction lies in the reported bin
    uv = oracle.oct_encode_many(r["dir"])
    assert (np.minimum((uv * N).astype(int), N - 1) == r["bin"].T).all()


def test_uniform_field_lambertian_closed_form():
    N, n = 32, 5000
    L = np.ones((1, N * N))
    nrm = np.tile(np.array([[0.0], [0.0], [1.0]], np.float32), (1, n))
    r = oracle.product_sample_fields(L, N, 11, 0, nrm=nrm, n=n)
    s = N // 8
    U, V = r["bin"][:, 0] // s, r["bin"][:, 1] // s
    a = (2 * U + 1) / 8.0 - 1.0
    b = (2 * V + 1) / 8.0 - 1.0
    zc = 1.0 - (np.abs(a) + np.abs(b)) ** 2
    assert (np.abs(a) + np.abs(b) < 1).all()           # only the 24 upper cells
    np.testing.assert_allclose(r["pdf"], zc / 15.0 * 64 / (4 * np.pi), rtol=1e-12)
    assert (r["dir"][2] >= 0).all()
    assert len(set(zip(U.tolist(), V.tolist()))) == 24


def test_constant_table_and_degenerate_normals_are_plain_guiding():
    N, n = 16, 300
    L = rand_fields(n, N, 5)
    plain = L / L.sum(1, keepdims=True) * (N * N) / (4 * np.pi)
    for kw in (dict(bsdf=np.ones((n, 64), np.float32)),
               dict(nrm=np.zeros((3, n), np.float32)),
               dict(nrm=np.full((3, n), np.nan, np.float32)),
               dict(nrm=np.full((3, n), np.inf, np.float32))):
        r = oracle.product_sample_fields(L, N, 2, 1, **kw)
        b = r["bin"][:, 1] * N + r["bin"][:, 0]
        np.testing.assert_allclose(r["pdf"], plain[np.arange(n), b], rtol=1e-12)


def test_n8_cell_is_the_bin():
    N, n = 8, 500
    L = rand_fields(n, N, 9)
    tab = np.random.default_rng(4).uniform(0, 1, (n, 64)).astype(np.float32)
    r = oracle.product_sample_fields(L, N, 3, 2, bsdf=tab)
    prod = L * tab
    b = r["bin"][:, 1] * 8 + r["bin"][:, 0]
    np.testing.assert_allclose(r["pdf"], (prod / prod.sum(1, keepdims=True))[np.arange(n), b] * 64 / (4 * np.pi),
                               rtol=1e-12)


def test_chi_square_of_one_field():
    from scipy.stats import chi2
    N, n = 16, 60000
    L = rand_fields(1, N, 21)
    nrm = np.tile(np.array([[0.3], [-0.5], [0.8]], np.float32), (1, n))
    r = oracle.product_sample_fields(L, N, 99, 4, nrm=nrm, n=n)
    p = direct_pdf(L, N, f32_cos_table(nrm[:, :1]))[0] * (4 * np.pi / (N * N))
    cnt = np.bincount(r["bin"][:, 1] * N + r["bin"][:, 0], minlength=N * N)
    assert cnt[p == 0].sum() == 0
    exp = p * n
    big = exp >= 5
    stat = (((cnt[big] - exp[big]) ** 2) / exp[big]).sum()
    rest = exp[~big & (p > 0)].sum()
    dof = big.sum() - 1
    if rest > 0:
        stat += (cnt[~big].sum() - rest) ** 2 / rest
        dof += 1
    assert chi2.sf(stat, dof) > 1e-4


@pytest.mark.parametrize("N", [8, 32])
def test_pdf_eval_normalized_and_consistent(N):
    n = 64
    L = rand_fields(n, N, 31)
    nrm = np.random.default_rng(2).normal(size=(3, n)).astype(np.float32)
    # sum over the bin centres of pdf * (4 pi / N^2) is one for every query
    cent = oracle.dir_table(N).reshape(N * N, 3).T.astype(np.float64)
    tot = np.zeros(n)
    for b in range(N * N):
        d = np.repeat(cent[:, b:b + 1], n, 1)
        tot += oracle.product_pdf_fields(L, N, d, nrm=nrm)
    np.testing.assert_allclose(tot * 4 * np.pi / (N * N), 1.0, rtol=1e-12)
    r = oracle.product_sample_fields(L, N, 5, 6, nrm=nrm)
    np.testing.assert_allclose(oracle.product_pdf_fields(L, N, r["dir"], nrm=nrm), r["pdf"], rtol=1e-12)


@pytest.fixture(scope="module")
def box(orc):
    rects = synth.cornell_box()
    o = orc.SVO(rects, 6)
    xyz, em = o.leaf_info()
    assert o.accumulate(*synth.leaf_splats(xyz, o.normals(6), em, 6, seed=2)) == 0
    o.propagate()
    pos, nrm, _ = synth.area_points(rects, 600, 5)
    return o, pos, nrm


def test_svo_product_uses_the_vertex_field(box):
    o, pos, nrm = box
    N = 16
    r = o.product_sample(pos, N, 4, 1, nrm=nrm)
    L, _ = o.field(pos, N)
    want = direct_pdf(L, N, f32_cos_table(nrm))
    b = r["bin"][:, 1] * N + r["bin"][:, 0]
    np.testing.assert_allclose(r["pdf"], want[np.arange(pos.shape[1]), b], rtol=1e-12)
    e = o.product_pdf_eval(pos, r["dir"].astype(np.float32), N, nrm=nrm)
    ok = e["edge"] > 1e-6
    np.testing.assert_allclose(e["pdf"][ok], r["pdf"][ok], rtol=1e-12)
    # surface points sample the hemisphere of their normal
    cos = (r["dir"] * nrm).sum(0)
    assert (cos > -0.2).all()


def test_binned_product_members_use_origin_field_and_own_normal(box):
    o, pos, nrm = box
    N = 16
    r = o.binned_sample(pos, 64, 3, N, 8, 2, nrm=nrm)
    org = r["origin"]
    uo = np.unique(org)
    fields = dict(zip(uo.tolist(), o.field(pos[:, uo], N)[0]))
    L = np.stack([fields[int(k)] for k in org])
    want = direct_pdf(L, N, f32_cos_table(nrm))
    b = r["bin"][:, 1] * N + r["bin"][:, 0]
    np.testing.assert_allclose(r["pdf"], want[np.arange(pos.shape[1]), b], rtol=1e-12)
