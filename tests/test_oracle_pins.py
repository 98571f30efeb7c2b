"""Pins of the CPU oracle against facts that do not come from its own code:
published known-answer vectors, closed forms, exact-rational brute force on
tiny grids, invariants and textbook routines (numpy/torch rounding, chi-square).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ helpers --
def morton_py(x, y, z, bits=10):
    """Morton key by string interleaving (z y x per bit, most significant first)."""
    bx, by, bz = (format(v, f"0{bits}b") for v in (x, y, z))
    return int("".join(bz[i] + by[i] + bx[i] for i in range(bits)), 2)


def rect(axis, c, lo, hi, sign=1, emissive=0):
    return synth.make_rect(axis, c, lo, hi, sign, emissive)


def rects(*rs):
    return np.array(list(rs), dtype=synth.RECT_DTYPE)


def closed_box():
    rs = []
    for a in range(3):
        rs.append(rect(a, 0.0, (0, 0), (1, 1), +1))
        rs.append(rect(a, 1.0, (0, 0), (1, 1), -1))
    return rects(*rs)


# --------------------------------------------------------------- Philox -----
def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox(v[0:4], v[4:6])
        assert list(out) == v[6:10]


# --------------------------------------------------------------- Morton -----
def test_morton_interleave(orc):
    rng = np.random.default_rng(0)
    for _ in range(500):
        x, y, z = (int(v) for v in rng.integers(0, 1024, 3))
        k = orc.morton(x, y, z)
        assert k == morton_py(x, y, z)
        assert k >> 3 == orc.morton(x >> 1, y >> 1, z >> 1)
        assert k & 7 == (x & 1) | ((y & 1) << 1) | ((z & 1) << 2)


# ------------------------------------------------------- octahedral map -----
@pytest.mark.parametrize("xy,d", [
    ((0.5, 0.5), (0, 0, 1)), ((0.0, 0.0), (0, 0, -1)), ((1.0, 1.0), (0, 0, -1)),
    ((0.0, 1.0), (0, 0, -1)), ((1.0, 0.0), (0, 0, -1)), ((1.0, 0.5), (1, 0, 0)),
    ((0.0, 0.5), (-1, 0, 0)), ((0.5, 1.0), (0, 1, 0)), ((0.5, 0.0), (0, -1, 0)),
])
def test_octahedral_special_points(orc, xy, d):
    np.testing.assert_allclose(orc.oct_decode(*xy), d, atol=1e-15)


def test_octahedral_roundtrip_and_unit(orc):
    rng = np.random.default_rng(1)
    v = rng.normal(size=(3, 20000))
    v /= np.linalg.norm(v, axis=0)
    xy = orc.oct_encode_many(v)
    assert xy.min() >= 0 and xy.max() <= 1
    back = orc.oct_decode_many(xy)
    np.testing.assert_allclose(back, v, atol=1e-12)
    sq = rng.random((2, 20000)) * 0.998 + 0.001
    d = orc.oct_decode_many(sq)
    np.testing.assert_allclose(np.linalg.norm(d, axis=0), 1.0, atol=1e-14)
    np.testing.assert_allclose(orc.oct_encode_many(d), sq, atol=1e-12)


@pytest.mark.parametrize("N", [8, 16])
def test_octahedral_equal_area_chi2(orc, N):
    """Uniform sphere directions land uniformly in the N x N bins (each bin is
    an equal solid-angle patch of 4*pi/N^2)."""
    rng = np.random.default_rng(2 + N)
    v = rng.normal(size=(3, 1 << 20))
    v /= np.linalg.norm(v, axis=0)
    xy = orc.oct_encode_many(v)
    u = np.minimum((xy[0] * N).astype(int), N - 1)
    w = np.minimum((xy[1] * N).astype(int), N - 1)
    h = np.bincount(w * N + u, minlength=N * N)
    p = stats.chisquare(h).pvalue
    assert p > 1e-3, p


@pytest.mark.parametrize("N", [8, 16, 32])
def test_dir_table_consistent(orc, N):
    t = orc.dir_table(N).astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(t, axis=1), 1.0, atol=2e-7)
    xy = orc.oct_encode_many(t.T)
    cu, cv = np.meshgrid((np.arange(N) + 0.5) / N, (np.arange(N) + 0.5) / N)
    np.testing.assert_allclose(xy[0], cu.ravel(), atol=2e-6)
    np.testing.assert_allclose(xy[1], cv.ravel(), atol=2e-6)


# --------------------------------------------------------- voxelization -----
def brute_cells(r, D):
    """Leaf keys covered by a rectangle, by exact-rational cell tests:
    along each in-plane axis the cells whose half-open extent meets the open
    interval (lo, hi) (or holds lo when lo == hi); along the plane axis the cell
    holding c. The last cell also holds the value 1."""
    R = 1 << D
    F = Fraction

    def holds(i, v):
        return (F(i, R) <= v < F(i + 1, R)) or (i == R - 1 and v == 1)

    def covered(i, lo, hi):
        if lo < hi:
            return F(i, R) < hi and F(i + 1, R) > lo
        return holds(i, lo)

    a = int(r["axis"])
    j0, j1 = [j for j in range(3) if j != a]
    c, lo0, lo1, hi0, hi1 = (F(float(v)) for v in
                             (r["c"], r["lo"][0], r["lo"][1], r["hi"][0], r["hi"][1]))
    A = [i for i in range(R) if holds(i, c)]
    B = [i for i in range(R) if covered(i, lo0, hi0)]
    Cc = [i for i in range(R) if covered(i, lo1, hi1)]
    keys = set()
    for ia in A:
        for ib in B:
            for ic in Cc:
                xyz = [0, 0, 0]
                xyz[a], xyz[j0], xyz[j1] = ia, ib, ic
                keys.add(morton_py(*xyz))
    return keys


def random_rects(rng, n, D, boundary_frac=0.4):
    R = 1 << D
    out = []
    for _ in range(n):
        def val():
            if rng.random() < boundary_frac:
                return float(np.float32(rng.integers(0, R + 1) / R))
            return float(np.float32(rng.random()))
        a = int(rng.integers(0, 3))
        c = val()
        l0, h0 = sorted([val(), val()])
        l1, h1 = sorted([val(), val()])
        if rng.random() < 0.1:
            h0 = l0
        out.append(rect(a, c, (l0, l1), (h0, h1), int(rng.choice([-1, 1]))))
    return rects(*out)


@pytest.mark.parametrize("D", [2, 3, 4, 5])
def test_voxelizer_vs_exact_brute_force(orc, D):
    rng = np.random.default_rng(10 + D)
    for trial in range(6):
        rs = random_rects(rng, 5, D)
        want = set()
        for r in rs:
            want |= brute_cells(r, D)
        s = orc.SVO(rs, D)
        got = set(int(k) for k in s.keys(D))
        assert got == want, (D, trial)
        # levels: unique parents of the level below
        for l in range(D - 1, -1, -1):
            assert set(int(k) for k in s.keys(l)) == set(int(k) >> 3 for k in s.keys(l + 1))


def test_cornell_level_closed_form(orc):
    gold = {}
    for line in open(os.path.join(GOLD, "cornell_levels.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            gold[k] = [int(x) for x in v]
    box = synth.cornell_box()
    walls = box[:5]
    s = orc.SVO(walls, 6)
    assert s.level_sizes() == gold["levels"]
    for l in range(2, 7):
        R = 1 << l
        assert s.level_size(l) == R ** 3 - (R - 2) * (R - 1) * (R - 2)
    s2 = orc.SVO(box, 6)
    _, em = s2.leaf_info()
    assert int(em.sum()) == gold["light_leaves"][0]


# --------------------------------------------------------------- k-means ----
def _leaf_normal(orc, rs, D=4):
    s = orc.SVO(rects(*rs), D)
    assert s.level_size(D) == 1
    return s.normals(D)[0]


def test_kmeans_single_wall(orc):
    for a in range(3):
        for sg in (-1, 1):
            s = orc.SVO(rects(rect(a, 0.3, (0.1, 0.2), (0.7, 0.9), sg)), 5)
            n = s.normals(5)
            want = np.zeros(3, np.float32)
            want[a] = sg
            assert (n == want).all()
            for l in range(5):  # inner nodes of a flat wall keep the normal
                assert (s.normals(l) == want).all()


def test_kmeans_opposite_normals_do_not_cancel(orc):
    p = 0.55
    for first in (1, -1):
        n = _leaf_normal(orc, [rect(0, p, (p, p), (p, p), first), rect(0, p, (p, p), (p, p), -first)])
        assert list(n) == [first, 0, 0]   # the seed's side, not a zero vector


def _ulp_close(x, want, ulps=1):
    x = np.float32(x)
    return abs(float(x) - want) <= ulps * float(np.spacing(np.float32(want)))


def test_kmeans_edge_and_corner(orc):
    p = 0.55
    n = _leaf_normal(orc, [rect(0, p, (p, p), (p, p), 1), rect(2, p, (p, p), (p, p), 1)])
    assert n[1] == 0 and n[0] == n[2] and _ulp_close(n[0], 1 / math.sqrt(2))
    n = _leaf_normal(orc, [rect(0, p, (p, p), (p, p), 1), rect(1, p, (p, p), (p, p), 1),
                           rect(2, p, (p, p), (p, p), 1)])
    assert n[0] == n[1] == n[2] and _ulp_close(n[0], 1 / math.sqrt(3))
    # +x, -x, +z: A = {+x, +z}, B = {-x} -> normalize(1, 0, 1)
    n = _leaf_normal(orc, [rect(0, p, (p, p), (p, p), 1), rect(0, p, (p, p), (p, p), -1),
                           rect(2, p, (p, p), (p, p), 1)])
    assert n[1] == 0 and n[0] == n[2] and _ulp_close(n[0], 1 / math.sqrt(2))


# ---------------------------------------------------------------- march -----
def brute_march(occ, D, O, q):
    """First occupied non-origin leaf by sorting every boundary-crossing event
    of the ray by (exact parameter, axis) and applying them in order."""
    S = 1 << (30 - D)
    R = 1 << D
    c0 = [O[j] >> (30 - D) for j in range(3)]
    ev = []
    for j in range(3):
        if q[j] > 0:
            for k in range(c0[j] + 1, R + 1):
                ev.append((Fraction(k * S - O[j], q[j]), j, 1, k * S))
        elif q[j] < 0:
            for k in range(c0[j], -1, -1):
                ev.append((Fraction(O[j] - k * S, -q[j]), j, -1, k * S))
    ev.sort(key=lambda e: (e[0], e[1]))
    c = list(c0)
    for t, j, sgn, B in ev:
        c[j] += sgn
        if not 0 <= c[j] < R:
            return dict(hit=0)
        k = morton_py(*c)
        if k in occ:
            return dict(hit=1, axis=j, key=k, delta=abs(B - O[j]))
    return dict(hit=0)


def _ray_cases(rng, D, n):
    R = 1 << D
    special = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, 0, -1), (1, 1, 0), (1, -1, 0), (-1, 1, 1),
               (1, 1, 1), (1, 2, 0), (2, 1, -1), (3, -1, 2)]
    for i in range(n):
        if rng.random() < 0.5:   # origin on cell corners / faces
            p = rng.integers(0, R + 1, 3) / R
            if rng.random() < 0.5:
                p[rng.integers(0, 3)] = rng.random()
        else:
            p = rng.random(3)
        p = np.clip(p, 0, 1).astype(np.float32)
        if rng.random() < 0.4:
            d = np.array(special[rng.integers(len(special))], np.float64)
            d *= rng.choice([-1, 1], 3)
        else:
            d = rng.normal(size=3)
        d = (d / np.linalg.norm(d)).astype(np.float32)
        yield p, d


@pytest.mark.parametrize("D", [3, 4])
def test_march_vs_event_sort_brute_force(orc, D):
    rng = np.random.default_rng(20 + D)
    for trial in range(8):
        rs = random_rects(rng, 4, D, boundary_frac=0.6)
        s = orc.SVO(rs, D)
        occ = set(int(k) for k in s.keys(D))
        for p, d in _ray_cases(rng, D, 150):
            O, q = orc.quantize(p, d)
            want = brute_march(occ, D, [int(v) for v in O], [int(v) for v in q])
            for hier in (False, True):
                got = s.march_one(p, d, hier=hier)
                assert got["hit"] == want["hit"], (p, d, hier)
                if want["hit"]:
                    assert (got["axis"], got["key"], got["delta"]) == \
                        (want["axis"], want["key"], want["delta"]), (p, d, hier)


def test_march_flat_equals_hierarchical_cornell(orc):
    box = synth.cornell_box()
    s = orc.SVO(box, 6)
    pos, _, _ = synth.area_points(box, 4096, 3)
    flat = s.debug_march(pos, 8, hier=False)
    hier = s.debug_march(pos, 8, hier=True)
    assert (flat == hier).all()
    assert flat[..., 0].mean() > 0.3


def test_march_flat_equals_hierarchical_room(orc):
    room = synth.room()
    s = orc.SVO(room, 10)
    pos, _, _ = synth.area_points(room, 96, 14)
    flat = s.debug_march(pos, 16, hier=False)
    hier = s.debug_march(pos, 16, hier=True)
    assert (flat == hier).all()


# ------------------------------------------------------------ footprint -----
def test_footprint_closed_form(orc):
    rows = [l.split()[:4] for l in open(os.path.join(GOLD, "footprint_cases.txt"))
            if l.strip() and not l.startswith("#")]
    D = 6
    for N, r, A, k in rows:
        N, r, A, k = int(N), float(r), float(A), int(k)
        assert abs(r * r * 4 * math.pi / N ** 2 - A) < 1e-4 * A
        # origin on the x=0 face (r integer) or at a leaf centre (r half-integer)
        ox = 0.0 if r == int(r) else 0.5
        wall = int(round(r + ox))
        s = orc.SVO(rects(rect(0, wall / 64, (0, 0), (1, 1), -1)), D)
        rec = s.eval_one([ox / 64, 0.5 + 0.25 / 64, 0.5 + 0.25 / 64], [1, 0, 0], N)
        assert rec["hit"] == 1 and rec["axis"] == 0
        assert rec["r"] == r
        assert rec["k"] == k, (N, r, rec)
        assert rec["node"] == rec["leaf"] >> (3 * k)


# ------------------------------------------- closed-form PDFs and invariants --
@pytest.mark.parametrize("D,N", [(4, 8), (5, 16), (6, 8), (5, 64), (4, 128)])
def test_uniform_enclosure(orc, D, N):
    s = orc.SVO(closed_box(), D)
    s.set_uniform_exitance(1.0)
    rng = np.random.default_rng(D)
    pos = rng.uniform(0.1, 0.9, (3, 64)).astype(np.float32)
    pdf = s.guide_pdf(pos, N)
    np.testing.assert_allclose(pdf, 1 / (4 * math.pi), rtol=1e-13)
    L, _ = s.field(pos, N)
    np.testing.assert_allclose(L, float(np.float32(1.0)) + float(np.float32(0.01)), rtol=1e-15)


def test_all_miss_is_uniform(orc):
    empty = np.zeros(0, synth.RECT_DTYPE)
    s = orc.SVO(empty, 5)
    assert s.level_sizes() == [0] * 6
    pos = np.random.default_rng(0).random((3, 16)).astype(np.float32)
    np.testing.assert_allclose(s.guide_pdf(pos, 8), 1 / (4 * math.pi), rtol=1e-13)
    # a point on the outer face of a single wall sees it only on one side
    s = orc.SVO(rects(rect(2, 0.5, (0, 0), (1, 1), 1)), 5)
    s.set_uniform_exitance(3.0)
    L, _ = s.field(np.array([[0.5], [0.5], [0.25]], np.float32), 8)
    t = orc.dir_table(8)
    up = t[:, 2] > 0
    assert (L[0, up] > 3.0).all() and np.allclose(L[0, ~up], float(np.float32(0.01)))


def _c1_svo(orc, fmt=0):
    box = synth.cornell_box()
    s = orc.SVO(box, 6)
    xyz, em = s.leaf_info()
    p, w, c = synth.leaf_splats(xyz, s.normals(6), em, 6, seed=2)
    assert s.accumulate(p, w, c) == 0
    s.propagate(fmt)
    return box, s


def test_pdf_normalized_and_mc_integral(orc):
    box, s = _c1_svo(orc)
    pos, _, _ = synth.area_points(box, 64, 3)
    for N in (8, 16):
        pdf = s.guide_pdf(pos, N)
        np.testing.assert_allclose(pdf.sum(1) * 4 * math.pi / N ** 2, 1.0, rtol=1e-12)
        assert (pdf > 0).all()
    # Monte-Carlo: E[4*pi*pdf(w)] over uniform w equals the integral of pdf
    rng = np.random.default_rng(5)
    M = 8192
    v = rng.normal(size=(3, M))
    v /= np.linalg.norm(v, axis=0)
    P = np.repeat(pos[:, :1], M, 1)
    r = s.pdf_eval(P, v.astype(np.float32), 8)
    x = 4 * math.pi * r["pdf"]
    assert abs(x.mean() - 1) < 3 * x.std() / math.sqrt(M) + 1e-9


def test_sampling_chi2(orc):
    box, s = _c1_svo(orc)
    pos, _, _ = synth.area_points(box, 8, 3)
    N = 8
    n = 1 << 16
    for vi in range(2):
        P = np.repeat(pos[:, vi:vi + 1], n, 1)
        out = s.guide_sample(P, N, seed=1234 + vi, bounce=0)
        pdf = s.guide_pdf(pos[:, vi:vi + 1], N)[0]
        prob = pdf * 4 * math.pi / N ** 2
        b = out["bin"][:, 1] * N + out["bin"][:, 0]
        h = np.bincount(b, minlength=N * N).astype(float)
        exp = prob * n
        order = np.argsort(exp)
        # merge bins with small expectation
        hs, es, acc_h, acc_e = [], [], 0.0, 0.0
        for i in order:
            acc_h += h[i]
            acc_e += exp[i]
            if acc_e >= 5:
                hs.append(acc_h); es.append(acc_e); acc_h = acc_e = 0.0
        if acc_e > 0:
            hs[-1] += acc_h; es[-1] += acc_e
        assert stats.chisquare(hs, es).pvalue > 1e-3
        np.testing.assert_allclose(out["pdf"], pdf[b], rtol=1e-14)
        # the continuous direction lies in its bin; sub-bin position uniform
        xy = orc.oct_encode_many(out["dir"])
        fu, fv = xy[0] * N - out["bin"][:, 0], xy[1] * N - out["bin"][:, 1]
        assert (fu > -1e-9).all() and (fu < 1 + 1e-9).all() and (fv > -1e-9).all() and (fv < 1 + 1e-9).all()
        sub = (fu >= 0.5).astype(int) * 2 + (fv >= 0.5)
        assert stats.chisquare(np.bincount(sub, minlength=4)).pvalue > 1e-3
        np.testing.assert_allclose(np.linalg.norm(out["dir"], axis=0), 1.0, atol=1e-12)


def test_pdf_eval_matches_sample_pdf(orc):
    box, s = _c1_svo(orc)
    pos, _, _ = synth.area_points(box, 256, 7)
    out = s.guide_sample(pos, 8, seed=9, bounce=3)
    ev = s.pdf_eval(pos, out["dir"].astype(np.float32), 8)
    ok = ev["edge"] > 1e-5
    assert ok.mean() > 0.99
    np.testing.assert_array_equal(ev["bin"][ok], out["bin"][ok])
    np.testing.assert_allclose(ev["pdf"][ok], out["pdf"][ok], rtol=1e-14)


# ------------------------------------------------------ splat / propagate ----
def test_one_splat_per_leaf_side_is_exact(orc):
    box, s = _c1_svo(orc)
    s32, s64, cnt = s.leaf_accum()
    assert (cnt == 1).all()
    e32, e64 = s.exitance(6)
    assert (e32.astype(np.float64) == e64).all()
    # grey RGB: the Rec.709 weights sum to one, so luminance == y within 2 ulp
    xyz, em = s.leaf_info()
    rng = np.random.default_rng(2)
    y = rng.lognormal(0.0, 1.0, size=(2, len(em)))
    y[:, em != 0] *= 100.0
    y = y.astype(np.float32).T
    assert (np.abs(e32 - y) <= 2 * np.spacing(y)).all()


def test_dropped_splats_counted(orc):
    box = synth.cornell_box()
    s = orc.SVO(box, 6)
    pos, nrm, _ = synth.area_points(box, 1000, 4)
    wo = nrm.copy()
    rgb = np.ones((3, 1000), np.float32)
    bad = np.zeros(1000, bool)
    pos[0, 0] = np.nan; bad[0] = True
    pos[1, 1] = 1.5; bad[1] = True
    rgb[2, 2] = np.inf; bad[2] = True
    rgb[:, 3] = -1.0; bad[3] = True
    wo[0, 4] = np.nan; bad[4] = True
    pos[:, 5] = 0.5; bad[5] = True       # empty interior leaf
    pos[0, 6] = -0.001; bad[6] = True
    d = s.accumulate(pos, wo, rgb)
    assert d == bad.sum() == s.dropped()
    _, _, cnt = s.leaf_accum()
    assert cnt.sum() == 1000 - bad.sum()


def test_uniform_exitance_propagates_exactly(orc):
    box = synth.cornell_box()
    s = orc.SVO(box, 6)
    xyz, em = s.leaf_info()
    p, w, _ = synth.leaf_splats(xyz, s.normals(6), em, 6)
    s.accumulate(p, w, np.ones_like(p))
    s.propagate()
    for l in range(7):
        e32, e64 = s.exitance(l)
        assert (e32 == 1.0).all() and (e64 == 1.0).all()


def test_propagate_closed_form_tiny_tree(orc):
    # depth 1: wall x=0 covers the four x=0 cells; y=0 cells face +x, y=1 cells -x
    rs = rects(rect(0, 0.0, (0, 0), (0.5, 1), +1), rect(0, 0.0, (0.5, 0), (1, 1), -1))
    s = orc.SVO(rs, 1)
    keys = s.keys(1)
    assert list(keys) == [0, 2, 4, 6]
    n = s.normals(1)
    assert (n[:, 0] == [1, -1, 1, -1]).all()
    # powers of two: grey luminance is then exact (the weights sum to one)
    vals = np.array([[1.0, 2.0], [4.0, 8.0], [16.0, 32.0], [64.0, 128.0]], np.float32)
    ctr = np.array([[0.25, 0.25, 0.25], [0.25, 0.75, 0.25], [0.25, 0.25, 0.75], [0.25, 0.75, 0.75]])
    P, W, Cc = [], [], []
    for i in range(4):
        for side, sg in ((0, 1.0), (1, -1.0)):
            P.append(ctr[i]); W.append(n[i] * sg); Cc.append([vals[i, side]] * 3)
    s.accumulate(np.array(P, np.float32).T, np.array(W, np.float32).T, np.array(Cc, np.float32).T)
    s.propagate()
    e32, e64 = s.exitance(0)
    assert list(s.normals(0)[0]) == [1, 0, 0]
    # root side 0 (+x) averages side 0 of +x children and side 1 of -x children
    want0 = (vals[0, 0] + vals[1, 1] + vals[2, 0] + vals[3, 1]) / 4
    want1 = (vals[0, 1] + vals[1, 0] + vals[2, 1] + vals[3, 0]) / 4
    assert e64[0, 0] == want0 and e64[0, 1] == want1
    assert e32[0, 0] == np.float32(want0) and e32[0, 1] == np.float32(want1)


# -------------------------------------------------- 16-bit storage formats ---
def test_fp16_bf16_rounding_vs_numpy_torch(orc):
    import torch
    rng = np.random.default_rng(3)
    x = np.concatenate([
        rng.lognormal(0, 6, 20000).astype(np.float32),
        -rng.lognormal(0, 6, 2000).astype(np.float32),
        np.float32(2.0) ** np.arange(-30, 20, dtype=np.float32),
        np.array([0.0, 65504.0, 65519.0, 65520.0, 1e6, 5.96e-8, 2.98e-8, 3e-8, np.inf], np.float32),
    ])
    # exact ties for binary16 and bfloat16
    ties16 = (np.arange(1, 200, dtype=np.float32) * 2 + 1) * np.float32(2.0 ** -11)
    ties_bf = (np.arange(1, 200, dtype=np.float32) * 2 + 1) * np.float32(2.0 ** -8) + 1
    x = np.concatenate([x, ties16, ties_bf]).astype(np.float32)
    want16 = x.astype(np.float16).astype(np.float32)
    got16 = orc.round_fmt(x, orc.FMT_FP16)
    assert np.array_equal(got16, want16)
    wantbf = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    gotbf = orc.round_fmt(x, orc.FMT_BF16)
    assert np.array_equal(gotbf, wantbf)
