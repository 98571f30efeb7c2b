"""Pins of the oracle's positional binning (Alg. 2, Partition-S) and per-bin
guiding (Alg. 3 with SelectOrigin).

The bins are checked against a direct definition written independently of
the bottom-up marking: a query's bin is the deepest node on its path with
level >= l_min whose subtree holds at least c_ray queries (the query's own
node counts), else its ancestor on level l_min. Closed forms: c_ray = 1 puts
every query in its own node; a c_ray above the queue length puts every query
in its level-l_min ancestor. Per-bin guiding: every member is sampled from
the field of its bin's origin, the origin is the member with the smallest
origin hash, and one bin's samples follow that field (chi-square).
"""
import collections

import numpy as np
import pytest

import synth


def morton_np(x, y, z, bits):
    k = np.zeros_like(x, dtype=np.int64)
    for i in range(bits):
        k |= ((x >> i) & 1) << (3 * i)
        k |= ((y >> i) & 1) << (3 * i + 1)
        k |= ((z >> i) & 1) << (3 * i + 2)
    return k


def query_nodes(o, pos, D):
    """(level, key) of the deepest existing node holding each quantized position."""
    q = np.clip(np.rint(pos.astype(np.float64) * 2.0 ** 30), 0, 2 ** 30 - 1).astype(np.int64)
    c = q >> (30 - D)
    key = morton_np(c[0], c[1], c[2], D)
    sets = [set(o.keys(l).tolist()) for l in range(D + 1)]
    lv = np.full(key.shape, -1)
    kk = np.zeros_like(key)
    for i in range(key.size):
        k, l = int(key[i]), D
        while l >= 0 and k not in sets[l]:
            k >>= 3
            l -= 1
        lv[i], kk[i] = l, k
    return lv, kk


def brute_bins(o, pos, D, c_ray, l_min):
    lv, kk = query_nodes(o, pos, D)
    cnt = collections.Counter()
    for l, k in zip(lv, kk):
        for m in range(l, -1, -1):
            cnt[(m, int(k) >> (3 * (l - m)))] += 1
    out = []
    for l, k in zip(lv, kk):
        b = (l, int(k))
        if l >= l_min:
            b = (l_min, int(k) >> (3 * (l - l_min)))
            for m in range(l, l_min - 1, -1):
                a = (m, int(k) >> (3 * (l - m)))
                if cnt[a] >= c_ray:
                    b = a
                    break
        out.append(b)
    return out


def as_keys(o, lv, ix):
    return [(int(l), int(o.keys(l)[i])) for l, i in zip(lv, ix)]


@pytest.fixture(scope="module")
def scene(orc):
    rects = synth.cornell_box()
    D = 6
    o = orc.SVO(rects, D)
    xyz, em = o.leaf_info()
    assert o.accumulate(*synth.leaf_splats(xyz, o.normals(D), em, D, seed=2)) == 0
    o.propagate()
    pos, nrm, _ = synth.area_points(rects, 3000, 7)
    # a few off-surface points (their leaf is empty: binned at an ancestor)
    extra = np.random.default_rng(8).uniform(0.3, 0.7, (3, 40)).astype(np.float32)
    pos = np.ascontiguousarray(np.concatenate([pos, extra], 1))
    return o, pos, D


@pytest.mark.parametrize("c_ray,l_min", [(1, 0), (8, 2), (64, 3), (300, 1), (5000, 4), (40, 6)])
def test_partition_matches_direct_definition(scene, c_ray, l_min):
    o, pos, D = scene
    lv, ix = o.partition(pos, c_ray, l_min)
    assert as_keys(o, lv, ix) == brute_bins(o, pos, D, c_ray, l_min)


def test_partition_closed_forms(scene):
    o, pos, D = scene
    nl, nk = query_nodes(o, pos, D)
    lv, ix = o.partition(pos, 1, 0)                  # every query is its own bin
    assert as_keys(o, lv, ix) == [(int(l), int(k)) for l, k in zip(nl, nk)]
    for l_min in (0, 2, 4):                          # nothing reaches c_ray: ancestors on l_min
        lv, ix = o.partition(pos, pos.shape[1] + 1, l_min)
        want = [(l_min, int(k) >> (3 * (l - l_min))) if l >= l_min else (int(l), int(k))
                for l, k in zip(nl, nk)]
        assert as_keys(o, lv, ix) == want
    lv, _ = o.partition(pos, 1, 0)
    assert (lv[:3000] == D).all()                    # surface points sit in occupied leaves
    assert (lv[3000:] < D).any()


def test_binned_members_sample_their_origin_field(orc, scene):
    o, pos, D = scene
    N, seed, bounce = 8, 21, 2
    r = o.binned_sample(pos, 64, 3, N, seed, bounce)
    org = r["origin"]
    assert (org >= 0).all()
    # the origin is a member of the bin, chosen by the smallest (hash, index)
    groups = collections.defaultdict(list)
    for i, (l, k) in enumerate(zip(r["level"], r["index"])):
        groups[(int(l), int(k))].append(i)
    for members in groups.values():
        h = [(int(orc.philox([i & 0xffffffff, i >> 32, bounce, 1], [seed & 0xffffffff, seed >> 32])[0]), i)
             for i in members]
        best = min(h)[1]
        assert all(org[i] == best for i in members)
    # every member's pdf is its origin field's pdf at the sampled bin
    uo = np.unique(org)
    fields = dict(zip(uo.tolist(), o.guide_pdf(pos[:, uo], N)))
    b = r["bin"]
    want = np.array([fields[int(org[i])][b[i, 1] * N + b[i, 0]] for i in range(pos.shape[1])])
    np.testing.assert_allclose(r["pdf"], want, rtol=1e-12)
    # each member keeps its own uniforms: samples differ within a bin
    first = groups[max(groups, key=lambda k: len(groups[k]))]
    assert len({tuple(np.round(r["dir"][:, i], 9)) for i in first}) == len(first)


def test_single_bin_chi_square(orc, scene):
    from scipy.stats import chi2
    o, pos, D = scene
    N = 8
    rng = np.random.default_rng(3)
    p = pos[:, rng.integers(0, 3000, 20000)]
    r = o.binned_sample(np.ascontiguousarray(p), 10 ** 9, 0, N, 5, 0)   # one bin: the root
    assert (r["level"] == 0).all() and len(np.unique(r["origin"])) == 1
    pdf = o.guide_pdf(p[:, r["origin"][:1]], N)[0]
    prob = pdf * (4 * np.pi / (N * N))
    cnt = np.bincount(r["bin"][:, 1] * N + r["bin"][:, 0], minlength=N * N)
    exp = prob * p.shape[1]
    big = exp >= 5
    stat = (((cnt - exp) ** 2) / exp)[big].sum()
    if (~big).any():
        stat += (cnt[~big].sum() - exp[~big].sum()) ** 2 / max(exp[~big].sum(), 1e-9)
    dof = big.sum() + (1 if (~big).any() else 0) - 1
    assert chi2.sf(stat, dof) > 1e-4
