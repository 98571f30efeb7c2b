"""Pins of three oracle decisions against facts outside its own code.

* Side of the field value (Sec. 3.2: every node keeps the exitance of both
  of its sides; Sec. 3.3: the node normal times the cone direction picks the
  value): a thin wall that sends different radiance from its two faces.
  Radiance leaving the upper face must reach every query above the wall and
  never one below it, whichever way the wall's normal points.
* Cone footprint (Eq. 7 and the ascent to the node whose area is closest to
  the disk's): golden rows in the intervals where the linear-area and the
  log-area readings of "closest" disagree, and the level of every hit of a
  random ray set against the direct argmin of |4^k - A|.
* Node-test count of the top-down traversal (the algorithmic bytes of the
  march): recounted here from the flat leaf sequence of the ray (exact
  rational event order) and the level occupancy sets, with no use of the
  oracle's hierarchical walk.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def morton_py(x, y, z, bits=10):
    bx, by, bz = (format(v, f"0{bits}b") for v in (x, y, z))
    return int("".join(bz[i] + by[i] + bx[i] for i in range(bits)), 2)


def rects(*rs):
    return np.array(list(rs), dtype=synth.RECT_DTYPE)


def rect(axis, c, lo, hi, sign=1):
    return synth.make_rect(axis, c, lo, hi, sign, 0)


EPS32 = float(np.float32(0.01))


# ----------------------------------------------------------- field side -----
def _two_sided_wall(orc, sign, D=5, up=4.0, down=2.0):
    """Wall z = 1/2 over the whole square; every leaf gets one splat of grey
    radiance `up` leaving along +z and one of `down` leaving along -z (grey
    values that are powers of two: their FP32 luminance and every mean of
    equal children are exact)."""
    s = orc.SVO(rects(rect(2, 0.5, (0, 0), (1, 1), sign)), D)
    xyz, _ = s.leaf_info()
    c = ((xyz.astype(np.float64) + 0.5) / (1 << D)).T.astype(np.float32)
    n = c.shape[1]
    wo_up = np.tile(np.array([[0], [0], [1]], np.float32), (1, n))
    pos = np.concatenate([c, c], 1)
    wo = np.concatenate([wo_up, -wo_up], 1)
    rgb = np.concatenate([np.full((3, n), up, np.float32), np.full((3, n), down, np.float32)], 1)
    assert s.accumulate(pos, wo, rgb) == 0
    s.propagate()
    return s


@pytest.mark.parametrize("sign", [1, -1])
def test_splat_side_follows_leaf_normal(orc, sign):
    """Splat rule as the interface states it: side 0 iff N_leaf . wo >= 0."""
    s = _two_sided_wall(orc, sign)
    s32, _, cnt = s.leaf_accum()
    assert (cnt == 1).all()
    want0 = 4.0 if sign > 0 else 2.0   # the splat leaving along +z has N . wo = sign
    assert (s32[:, 0] == want0).all() and (s32[:, 1] == 6.0 - want0).all()


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("N", [8, 16])
def test_field_sees_the_face_toward_the_query(orc, sign, N):
    s = _two_sided_wall(orc, sign)
    t = orc.dir_table(N)
    for zq, seen in ((0.75, 4.0), (0.25, 2.0)):
        p = np.array([[0.5 + 0.3 / 32], [0.5 + 0.3 / 32], [zq]], np.float32)
        L, _ = s.field(p, N)
        rec = s.debug_march(p, N)[0]
        hit = rec[:, 0] == 1
        toward = t[:, 2] * (0.5 - zq) > 0          # bin directions facing the wall
        assert hit.sum() > N * N // 4
        assert not (hit & ~toward).any()
        assert (L[0, hit] == seen + EPS32).all(), (sign, zq, np.unique(L[0, hit]))
        assert (L[0, ~hit] == EPS32).all()


# ------------------------------------------------------------ footprint -----
def _footprint_rows():
    rows = []
    for line in open(os.path.join(GOLD, "footprint_cases.txt")):
        if line.strip() and not line.startswith("#"):
            N, r, A, k = line.split()[:4]
            rows.append((int(N), float(r), float(A), int(k)))
    return rows


def _wall_hit(orc, r, N, D=6):
    """One hit at distance r (integer: origin on the x = 0 face; half-integer:
    origin at a leaf centre) along +x."""
    ox = 0.0 if r == int(r) else 0.5
    wall = int(round(r + ox))
    s = orc.SVO(rects(rect(0, wall / 64, (0, 0), (1, 1), -1)), D)
    return s.eval_one([ox / 64, 0.5 + 0.25 / 64, 0.5 + 0.25 / 64], [1, 0, 0], N)


def test_golden_rows_separate_linear_from_log_area():
    """Every interval (2 * 4^(k-1), 2.5 * 4^(k-1)] where the readings differ,
    k = 1, 2, 3, holds a golden row at N = 8 and the first two at N = 16."""
    rows = _footprint_rows()
    gaps = {(N, k) for (N, r, A, kk) in rows for k in range(1, 5)
            if 2 * 4 ** (k - 1) < A <= 2.5 * 4 ** (k - 1)}
    assert {(8, 1), (8, 2), (8, 3), (16, 1), (16, 2)} <= gaps


def test_golden_rows_are_the_linear_argmin():
    """The k of every golden row minimises |4^k - A| (ties to the finer k)."""
    for N, r, A, k in _footprint_rows():
        assert abs(r * r * 4 * math.pi / N ** 2 - A) < 1e-4 * A
        dist = [abs(4.0 ** j - A) for j in range(0, 8)]
        assert k == min(range(8), key=lambda j: (dist[j], j)), (N, r, A)


def test_footprint_golden_rows(orc):
    for N, r, A, k in _footprint_rows():
        rec = _wall_hit(orc, r, N)
        assert rec["hit"] == 1 and rec["axis"] == 0 and rec["r"] == r
        assert rec["k"] == k, (N, r, A, rec["k"])


def test_footprint_is_linear_argmin_on_random_hits(orc):
    """Over random rays in a random scene at depth 10, the oracle's level is
    argmin_k |4^k - A| with A recomputed from the record in FP32 (Eq. 7), and
    the sample covers the intervals where the log-area reading differs."""
    rng = np.random.default_rng(77)
    room = synth.room()
    s = orc.SVO(room, 10)
    pos, _, _ = synth.area_points(room, 40, 5)
    in_gap = 0
    for N in (8, 16, 32):
        om = np.float32(4 * math.pi / (N * N))
        t = orc.dir_table(N)
        recs = s.debug_march(pos, N)
        for i in range(pos.shape[1]):
            for b in np.nonzero(recs[i, :, 0] == 1)[0][::3]:
                rec = recs[i, b]
                axis, delta, k = int(rec[1]), int(rec[3]), int(rec[4])
                r = np.float32(np.float32(delta) * np.float32(2.0 ** -20)) / np.float32(abs(t[b, axis]))
                A = float(np.float32(np.float32(r * r) * om))
                want = min(range(11), key=lambda j: (abs(4.0 ** j - A), j))
                assert k == want, (N, i, b, A, k)
                in_gap += any(2 * 4 ** (j - 1) < A <= 2.5 * 4 ** (j - 1) for j in range(1, 11))
    assert in_gap > 200


def test_footprint_threshold_ties_cannot_occur():
    """A = (r r) omega in FP32 never equals a threshold 2.5 * 4^(j-1) for the
    field sizes used: the one FP32 product that rounds to each threshold is
    not the square of an FP32 value, so the tie rule (finer level) is never
    exercised and cannot be pinned by a hit."""
    f = np.float32
    for N in (8, 16, 32, 64, 128):
        om = f(4 * np.pi / (N * N))
        for j in range(1, 11):
            thr = f(2.5 * 4 ** (j - 1))
            s = f(float(thr) / float(om))
            for _ in range(40):
                s = np.nextafter(s, f(0))
            for _ in range(80):
                s = np.nextafter(s, f(np.inf))
                if f(s * om) != thr:
                    continue
                d = f(np.sqrt(float(s)))
                for dd in (np.nextafter(d, f(0)), d, np.nextafter(d, f(np.inf))):
                    assert f(dd * dd) != s, (N, j)


# ------------------------------------------------------- node-test count -----
def leaf_sequence(D, O, q):
    """Leaf cells of the ray O + t q from the origin's leaf on, in the order of
    their exact entry parameter (crossings of several axes at one parameter
    stepped lowest axis first), up to the cell that leaves the cube (None)."""
    S = 1 << (30 - D)
    R = 1 << D
    c0 = [O[j] >> (30 - D) for j in range(3)]
    ev = []
    for j in range(3):
        if q[j] > 0:
            ev += [(Fraction(k * S - O[j], q[j]), j, 1) for k in range(c0[j] + 1, R + 1)]
        elif q[j] < 0:
            ev += [(Fraction(O[j] - k * S, -q[j]), j, -1) for k in range(c0[j], -1, -1)]
    ev.sort(key=lambda e: (e[0], e[1]))
    seq = [tuple(c0)]
    c = list(c0)
    for _, j, sg in ev:
        c[j] += sg
        if not 0 <= c[j] < R:
            seq.append(None)
            return seq
        seq.append(tuple(c))
    return seq


def recount_tests(occ, D, O, q, count_from):
    """Node tests at levels >= count_from of the minimal top-down traversal:
    the origin's path is tested from the root down to its first empty level
    (or its leaf, which is left as the origin); then, for each leaf cell of
    the ray that lies outside the current empty cell, the levels below the
    deepest ancestor it shares with that cell are tested, down to the first
    empty level (the new current cell) or an occupied leaf (the hit)."""
    seq = leaf_sequence(D, O, q)

    def anc(c, l):
        return tuple(x >> (D - l) for x in c)

    def is_occ(l, c):
        return morton_py(*anc(c, l)) in occ[l]

    tests = 0
    c0 = seq[0]
    for l in range(D + 1):
        tests += l >= count_from
        if not is_occ(l, c0):
            cur = (l, anc(c0, l))
            break
    else:
        cur = (D, c0)
    for c in seq[1:]:
        if c is None:
            return tests, False
        lc, ac = cur
        if anc(c, lc) == ac:
            continue
        shared = max(m for m in range(lc + 1) if anc(c, m) == tuple(x >> (lc - m) for x in ac))
        for l in range(shared + 1, D + 1):
            tests += l >= count_from
            if not is_occ(l, c):
                cur = (l, anc(c, l))
                break
        else:
            return tests, True
    raise AssertionError("leaf sequence ended inside the cube")


@pytest.mark.parametrize("D", [3, 4, 5, 6])
def test_node_test_count_recount(orc, D):
    rng = np.random.default_rng(300 + D)
    if D == 6:
        scene = synth.cornell_box()
        pos, _, _ = synth.area_points(scene, 6, 3)
        N = 8
    else:
        import test_oracle_pins as tp
        scene = tp.random_rects(rng, 6, D, boundary_frac=0.5)
        pos = rng.random((3, 6)).astype(np.float32)
        pos[:, :2] = (rng.integers(0, (1 << D) + 1, (3, 2)) / (1 << D)).astype(np.float32)
        N = 8
    s = orc.SVO(scene, D)
    occ = [set(int(k) for k in s.keys(l)) for l in range(D + 1)]
    t = orc.dir_table(N)
    checked = 0
    for cf in (0, 2, 5):
        rec, vis = s.debug_march(pos, N, lds_levels=cf, visits=True)
        for i in range(pos.shape[1]):
            for b in range(0, N * N, 2 if D == 6 else 1):
                O, q = orc.quantize(pos[:, i], t[b])
                n_tests, hit = recount_tests(occ, D, [int(v) for v in O], [int(v) for v in q], cf)
                assert hit == bool(rec[i, b, 0]), (D, i, b)
                assert vis[i, b] == n_tests, (D, cf, i, b, vis[i, b], n_tests)
                checked += 1
    assert checked > 500
