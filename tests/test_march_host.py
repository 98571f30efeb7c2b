"""The library's traversal core (march_core.h), compiled for the host with
g++, against the oracle: every (vertex, bin) record bit-exact. This checks
the exact logic the gfx950 kernels run without needing a GPU."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def host_lib(tmp_path_factory):
    out = tmp_path_factory.mktemp("host") / "march_host.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
                           "-ffp-contract=off", os.path.join(HERE, "host", "march_host.cpp"),
                           "-o", str(out)])
    L = C.CDLL(str(out))
    L.host_debug_march.restype = None
    L.host_footprint_levels.restype = C.c_int
    L.host_footprint_levels.argtypes = [C.c_uint32, C.c_float, C.c_int, C.c_float]
    L.host_march_dirs.restype = None
    L.host_march_dirs.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p]
    L.host_first_step_dirs.restype = None
    L.host_first_step_dirs.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_int,
                                       C.c_void_p]
    L.host_debug_march.argtypes = [C.c_void_p] * 4 + [C.c_int, C.c_void_p, C.c_int64,
                                                       C.c_void_p, C.c_int, C.c_float,
                                                       C.c_void_p, C.c_void_p]
    return L


def level_words(l):
    return 1 if l <= 2 else 1 << (3 * l - 6)


def bitmaps_from_oracle(o, D):
    """Dense per-level bitmaps + per-word ranks (global node index), built
    from the oracle's sorted level keys."""
    woff = np.cumsum([0] + [level_words(l) for l in range(D + 1)])
    bits = np.zeros(woff[-1], np.uint64)
    rank = np.zeros(woff[-1], np.uint32)
    noff = np.zeros(12, np.int64)
    nrm = []
    base = 0
    for l in range(D + 1):
        k = o.keys(l).astype(np.int64)
        noff[l] = base
        np.bitwise_or.at(bits, woff[l] + (k >> 6), (np.uint64(1) << (k & 63).astype(np.uint64)))
        words = bits[woff[l]:woff[l + 1]]
        pc = np.array([bin(int(x)).count("1") for x in words], np.int64) if len(words) < 5000 else \
            np.unpackbits(words.view(np.uint8)).reshape(-1, 64).sum(1)
        rank[woff[l]:woff[l + 1]] = (base + np.concatenate([[0], np.cumsum(pc)[:-1]])).astype(np.uint32)
        base += len(k)
        nrm.append(o.normals(l))
    noff[D + 1:] = base
    return bits, rank, noff, np.ascontiguousarray(np.concatenate(nrm, 0))


def run_host(L, o, D, pos, N):
    import paper_2405_06997_amd as w   # host table only (no device work)
    bits, rank, noff, nrm = bitmaps_from_oracle(o, D)
    pos = np.ascontiguousarray(pos, np.float32)
    n = pos.shape[1]
    tab = np.ascontiguousarray(w.dir_table(N))
    out = np.zeros((n, N * N, 8), np.int32)
    vis = np.zeros((n, N * N), np.int32)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    L.host_debug_march(p(bits), p(rank), p(noff), p(nrm), D, p(pos), n, p(tab), N,
                       float(np.float32(4 * np.pi / (N * N))), p(out), p(vis))
    return out.astype(np.int64), vis.astype(np.int64)


def compare(orc_svo, got, gvis, pos, N):
    want, wvis = orc_svo.debug_march(pos, N, lds_levels=5, hier=False, visits=True)
    hit = want[..., 0] == 1
    assert np.array_equal(got[..., 0], want[..., 0])
    assert np.array_equal(got[hit], want[hit])
    assert np.array_equal(gvis, wvis)


@pytest.mark.parametrize("N", [8, 16])
def test_host_core_cornell(orc, host_lib, N):
    box = synth.cornell_box()
    o = orc.SVO(box, 6)
    pos, _, _ = synth.area_points(box, 2048, 3)
    got, vis = run_host(host_lib, o, 6, pos, N)
    compare(o, got, vis, pos, N)


def test_host_core_boundaries(orc, host_lib):
    """Query points on cell corners, faces and the cube's faces (p = 0, 1)."""
    box = synth.cornell_box()
    o = orc.SVO(box, 5)
    rng = np.random.default_rng(3)
    pos = (rng.integers(0, 33, (3, 1500)) / 32.0).astype(np.float32)
    pos[:, :500] = np.where(rng.random((3, 500)) < 0.5, pos[:, :500], rng.random((3, 500)))
    got, vis = run_host(host_lib, o, 5, pos, 8)
    compare(o, got, vis, pos, 8)


@pytest.mark.parametrize("D", [1, 2, 3, 4])
def test_host_core_shallow(orc, host_lib, D):
    """Depths below the first counted level (5): an occupied origin leaf adds
    no node test, as in the oracle's walk."""
    box = synth.cornell_box()
    o = orc.SVO(box, D)
    pos, _, _ = synth.area_points(box, 512, 3)
    got, vis = run_host(host_lib, o, D, pos, 8)
    assert (vis == 0).all()
    compare(o, got, vis, pos, 8)


def test_host_core_room(orc, host_lib):
    room = synth.room()
    o = orc.SVO(room, 10)
    cam, _, _ = synth.camera_queue(room)
    idx = np.random.default_rng(0).choice(cam.shape[1], 96, replace=False)
    rnd, _, _ = synth.area_points(room, 96, 14)
    pos = np.concatenate([cam[:, idx], rnd], 1)
    got, vis = run_host(host_lib, o, 10, pos, 16)
    compare(o, got, vis, pos, 16)


def test_host_core_special_directions(orc, host_lib):
    """Directions with zero components (the axes, the face and cube
    diagonals) and random ones, from points on cell corners, faces and the
    cube's faces, where the membership of points on planes decides: every
    (hit, axis, leaf key, |B - O|) equal to the oracle's single-ray march."""
    import itertools
    box = synth.cornell_box()
    D = 5
    o = orc.SVO(box, D)
    dirs = [np.array(v, float) / np.linalg.norm(v) for v in itertools.product([-1, 0, 1], repeat=3) if any(v)]
    rng = np.random.default_rng(8)
    r = rng.normal(size=(24, 3))
    r[np.arange(24), rng.integers(0, 3, 24)] = 0.0
    dirs += list(r / np.linalg.norm(r, axis=1, keepdims=True))
    dirs = np.ascontiguousarray(np.array(dirs, np.float32))
    pos = (rng.integers(0, 2 ** D + 1, (3, 160)) / 2 ** D).astype(np.float32)
    pos[:, 80:] = np.where(rng.random((3, 80)) < 0.5, pos[:, 80:], rng.random((3, 80))).astype(np.float32)
    # the corners of the 1/4 and 1/8 grids lie on the planes of many levels at
    # once, also in empty space, where a coarse cell is left through a face
    # the point lies on and the next cell is descended from that crossing
    g4 = np.stack(np.meshgrid(*[np.arange(5) / 4] * 3, indexing="ij")).reshape(3, -1)
    g8 = np.stack(np.meshgrid(*[np.arange(9) / 8] * 3, indexing="ij")).reshape(3, -1)
    pos = np.ascontiguousarray(np.concatenate([pos, g4, g8], 1).astype(np.float32))
    bits, _, _, _ = bitmaps_from_oracle(o, D)
    out = np.zeros((pos.shape[1], len(dirs), 4), np.int64)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    host_lib.host_march_dirs(p(bits), D, p(pos), pos.shape[1], p(dirs), len(dirs), p(out))
    hits = 0
    for i in range(pos.shape[1]):
        for b in range(len(dirs)):
            w = o.march_one(pos[:, i], dirs[b])
            got = out[i, b]
            assert got[0] == w["hit"], (i, b, got, w)
            if w["hit"]:
                hits += 1
                assert (got[1], got[2], got[3]) == (w["axis"], w["key"], w["delta"]), (i, b, got, w)
    assert hits > 1000


def test_host_first_step_from_neighbours(orc, host_lib):
    """The first step of a ray from an occupied origin leaf taken from the
    occupancy of the leaf's six face neighbours (the kernels' shortcut when
    no node-test count is kept): a hit is the oracle's hit (same leaf, axis
    and |B - O|), a miss the oracle's miss, and a ray sent on is one the
    oracle does not end in the empty neighbour it entered; the same step
    taken with no march state (first_leaf, first_exit) agrees. Camera-queue and
    area points of the room at depth 8 and points on the planes of many
    levels, with axis, diagonal and random directions."""
    import itertools
    room = synth.room()
    D = 8
    o = orc.SVO(room, D)
    dirs = [np.array(v, float) / np.linalg.norm(v) for v in itertools.product([-1, 0, 1], repeat=3) if any(v)]
    rng = np.random.default_rng(19)
    r = rng.normal(size=(40, 3))
    r[np.arange(20), rng.integers(0, 3, 20)] = 0.0
    dirs += list(r / np.linalg.norm(r, axis=1, keepdims=True))
    dirs = np.ascontiguousarray(np.array(dirs, np.float32))
    cam, _, _ = synth.camera_queue(room)
    area, _, _ = synth.area_points(room, 60, 23)
    # area points snapped to leaf corners: on the planes of every level below
    snap = np.clip(np.round(area[:, :30] * 2 ** D) / 2 ** D, 0, 1)
    pos = np.concatenate([cam[:, rng.choice(cam.shape[1], 60, replace=False)], area, snap], 1)
    pos = np.ascontiguousarray(pos.astype(np.float32))
    bits, _, _, _ = bitmaps_from_oracle(o, D)
    out = np.zeros((pos.shape[1], len(dirs), 4), np.int64)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    host_lib.host_first_step_dirs(p(bits), D, p(pos), pos.shape[1], p(dirs), len(dirs), p(out))
    seen = {0: 0, 1: 0, 2: 0}
    for i in range(pos.shape[1]):
        for b in range(len(dirs)):
            got = out[i, b]
            assert got[0] != -2, (i, b)   # the state-free form of the step agrees
            if got[0] < 0:
                continue
            seen[int(got[0])] += 1
            w = o.march_one(pos[:, i], dirs[b])
            if got[0] == 1:
                assert w["hit"] and (got[1], got[2], got[3]) == (w["axis"], w["key"], w["delta"]), (i, b, got, w)
            elif got[0] == 2:
                assert not w["hit"], (i, b, got, w)
            else:
                assert not (w["hit"] and w["key"] == got[2]), (i, b, got, w)
    assert seen[1] > 2000 and seen[0] > 500 and seen[2] > 0, seen


def test_host_footprint_levels_at_thresholds(host_lib):
    """Eq. 7: the footprint is k levels above the leaf, k the number of
    j = 1..D with A > 2.5 * 4^(j-1). With delta = 2^(30-D) and |d| = 1 the
    distance is exactly one leaf, so A = omega: every threshold, its FP32
    neighbours on both sides, 0, infinity and random values, for every D."""
    thr = [np.float32(2.5) * np.float32(4) ** j for j in range(12)]
    vals = [np.float32(0), np.float32(np.inf), np.float32(1e-30), np.float32(3e38)]
    for t in thr:
        t = np.float32(t)
        vals += [t, np.nextafter(t, np.float32(0)), np.nextafter(t, np.float32(np.inf)),
                 np.float32(t * np.float32(1.5))]
    vals += list(np.random.default_rng(4).uniform(0, 6e6, 300).astype(np.float32))
    for D in range(1, 11):
        for A in vals:
            want = sum(1 for j in range(1, D + 1) if A > np.float32(2.5) * np.float32(4) ** (j - 1))
            got = host_lib.host_footprint_levels(1 << (30 - D), 1.0, D, float(A))
            assert got == want, (D, float(A), got, want)
