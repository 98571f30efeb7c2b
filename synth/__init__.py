"""Seeded synthetic inputs for the path-guiding hot path.

This module only draws scenes, query-vertex queues and exitance splats. It
holds none of the guiding method's arithmetic (no voxelization, no traversal,
no octahedral map, no PDF): both the CPU oracle and the GPU library consume its
arrays unchanged.

The paper's scenes (Cornell Box, Sponza, Veach Door, Bathroom; Tab. 1 and
Sec. 5) are not available, so procedural stand-ins of the same kind are used:

* ``cornell_box``  -- unit cube, five diffuse walls (front face y=0 open), an
  emissive 0.2 x 0.2 ceiling quad and two axis-aligned boxes on the floor.
* ``room``         -- closed unit room, 64 random boxes and three 0.1 x 0.1
  area lights (one on the ceiling, two on side walls).

Rectangles are returned as a structured numpy array with the field layout of
``wfpg_rect`` in ``include/wfpg.h``: an axis-aligned rectangle lies in the plane
``x[axis] == c`` and spans ``[lo[k], hi[k]]`` along the other two axes taken in
increasing order; its normal is ``sign * e_axis``.
"""
from __future__ import annotations

import numpy as np

RECT_DTYPE = np.dtype([
    ("axis", "<i4"), ("c", "<f4"), ("lo", "<f4", (2,)), ("hi", "<f4", (2,)),
    ("sign", "<i4"), ("emissive", "<i4"),
])
assert RECT_DTYPE.itemsize == 32


def _other_axes(axis: int) -> tuple[int, int]:
    return tuple(j for j in range(3) if j != axis)  # type: ignore[return-value]


def make_rect(axis, c, lo, hi, sign, emissive=0):
    r = np.zeros((), RECT_DTYPE)
    r["axis"], r["c"], r["lo"], r["hi"] = axis, c, lo, hi
    r["sign"], r["emissive"] = sign, emissive
    return r


def _box_faces(lo3, hi3):
    """Six outward-facing rectangles of the axis-aligned box [lo3, hi3]."""
    out = []
    for a in range(3):
        j0, j1 = _other_axes(a)
        lo = (lo3[j0], lo3[j1])
        hi = (hi3[j0], hi3[j1])
        out.append(make_rect(a, lo3[a], lo, hi, -1))
        out.append(make_rect(a, hi3[a], lo, hi, +1))
    return out


def cornell_box(seed: int = 1) -> np.ndarray:
    """Tiny Cornell box: 5 walls with inward normals, 0.2x0.2 light, 2 boxes.

    Boxes have x/y extents U[0.15, 0.35] and z extent U[0.2, 0.6], rest on the
    floor and are placed without overlapping footprints by rejection sampling.
    """
    rng = np.random.default_rng(seed)
    rects = [
        make_rect(0, 0.0, (0, 0), (1, 1), +1),   # left   x=0
        make_rect(0, 1.0, (0, 0), (1, 1), -1),   # right  x=1
        make_rect(1, 1.0, (0, 0), (1, 1), -1),   # back   y=1
        make_rect(2, 0.0, (0, 0), (1, 1), +1),   # floor  z=0
        make_rect(2, 1.0, (0, 0), (1, 1), -1),   # ceiling z=1
        make_rect(2, 1.0, (0.4, 0.4), (0.6, 0.6), -1, emissive=1),  # light
    ]
    placed = []
    while len(placed) < 2:
        ext = np.array([rng.uniform(0.15, 0.35), rng.uniform(0.15, 0.35),
                        rng.uniform(0.2, 0.6)])
        lo = np.array([rng.uniform(0.0, 1.0 - ext[0]),
                       rng.uniform(0.0, 1.0 - ext[1]), 0.0])
        hi = lo + ext
        ok = all(hi[0] <= p[0][0] or p[1][0] <= lo[0] or
                 hi[1] <= p[0][1] or p[1][1] <= lo[1] for p in placed)
        if ok:
            placed.append((lo, hi))
    for lo, hi in placed:
        rects += _box_faces(lo.astype(np.float32), hi.astype(np.float32))
    return np.array(rects, dtype=RECT_DTYPE)


def room(seed_boxes: int = 11, seed_lights: int = 12, n_boxes: int = 64) -> np.ndarray:
    """Closed unit room with ``n_boxes`` random boxes and three area lights.

    Boxes: per-axis extents U[0.03, 0.10], centres U[0.05, 0.95]^3, overlaps
    allowed. Lights: 0.1 x 0.1 quads, one on the ceiling and two on two
    distinct side walls, each facing into the room.
    """
    rects = []
    for a in range(3):  # six walls, normals into the room
        rects.append(make_rect(a, 0.0, (0, 0), (1, 1), +1))
        rects.append(make_rect(a, 1.0, (0, 0), (1, 1), -1))
    rl = np.random.default_rng(seed_lights)
    # ceiling light
    x0, y0 = rl.uniform(0.1, 0.8, size=2)
    rects.append(make_rect(2, 1.0, (x0, y0), (x0 + 0.1, y0 + 0.1), -1, emissive=1))
    walls = rl.choice(4, size=2, replace=False)
    for w in walls:  # w -> (axis, c, sign)
        axis, c, sign = [(0, 0.0, +1), (0, 1.0, -1), (1, 0.0, +1), (1, 1.0, -1)][int(w)]
        u0 = rl.uniform(0.1, 0.8)
        v0 = rl.uniform(0.3, 0.8)  # second "other" axis is z for x/y walls
        rects.append(make_rect(axis, c, (u0, v0), (u0 + 0.1, v0 + 0.1), sign, emissive=1))
    rb = np.random.default_rng(seed_boxes)
    for _ in range(n_boxes):
        ext = rb.uniform(0.03, 0.10, size=3)
        ctr = rb.uniform(0.05, 0.95, size=3)
        lo = np.clip(ctr - ext / 2, 0.0, 1.0).astype(np.float32)
        hi = np.clip(ctr + ext / 2, 0.0, 1.0).astype(np.float32)
        rects += _box_faces(lo, hi)
    return np.array(rects, dtype=RECT_DTYPE)


def _rect_areas(rects: np.ndarray) -> np.ndarray:
    ext = (rects["hi"].astype(np.float64) - rects["lo"].astype(np.float64))
    return ext[:, 0] * ext[:, 1]


def area_points(rects: np.ndarray, n: int, seed: int):
    """``n`` points uniform by area over all rectangles.

    Returns (pos, nrm, rect_index): pos and nrm are SoA float32 arrays of shape
    (3, n); nrm is the rectangle normal.
    """
    rng = np.random.default_rng(seed)
    area = _rect_areas(rects)
    idx = rng.choice(len(rects), size=n, p=area / area.sum())
    r = rects[idx]
    uv = rng.random((n, 2))
    pos = np.empty((3, n), np.float64)
    nrm = np.zeros((3, n), np.float32)
    for a in range(3):
        m = r["axis"] == a
        j0, j1 = _other_axes(a)
        lo = r["lo"][m].astype(np.float64)
        hi = r["hi"][m].astype(np.float64)
        pos[a, m] = r["c"][m]
        pos[j0, m] = lo[:, 0] + uv[m, 0] * (hi[:, 0] - lo[:, 0])
        pos[j1, m] = lo[:, 1] + uv[m, 1] * (hi[:, 1] - lo[:, 1])
        nrm[a, m] = r["sign"][m]
    return np.ascontiguousarray(pos.astype(np.float32)), nrm, idx.astype(np.int64)


def camera_queue(rects: np.ndarray, width: int = 1920, height: int = 1080,
                 eye=(0.5, 0.02, 0.5), vfov_deg: float = 60.0, jitter_seed: int | None = None):
    """Primary hits of a pinhole camera looking along +y (z up), one ray per
    pixel centre (or, with ``jitter_seed``, per point uniform inside the pixel),
    intersected analytically against the rectangles in FP64.

    Each rectangle is only tested against the pixels inside the bounding box
    of its projection (all of them when it straddles the eye plane). Returns
    (pos, nrm, rect_index) in pixel order (rows top to bottom); pixels that hit
    nothing are removed (none inside a closed room).
    """
    eye = np.asarray(eye, np.float64)
    th = np.tan(np.radians(vfov_deg) / 2)
    aspect = width / height
    if jitter_seed is None:
        jx = np.full((height, width), 0.5)
        jy = jx
    else:
        rng = np.random.default_rng(jitter_seed)
        jx = rng.random((height, width))
        jy = rng.random((height, width))
    sx = (np.arange(width)[None, :] + jx) / width * 2 - 1
    sy = 1 - (np.arange(height)[:, None] + jy) / height * 2
    X = sx * aspect * th                            # (H, W)
    Z = sy * th
    inv = 1.0 / np.sqrt(X * X + 1.0 + Z * Z)
    D = np.stack([X * inv, inv, Z * inv], 0)       # (3, H, W) unit directions
    best_t = np.full((height, width), np.inf)
    best_r = np.full((height, width), -1, np.int64)
    for ri in range(len(rects)):
        r = rects[ri]
        a = int(r["axis"])
        j0, j1 = _other_axes(a)
        corners = []
        for u in (r["lo"][0], r["hi"][0]):
            for v in (r["lo"][1], r["hi"][1]):
                p = np.zeros(3)
                p[a], p[j0], p[j1] = r["c"], u, v
                corners.append(p)
        corners = np.array(corners) - eye
        depth = corners[:, 1]
        if np.all(depth <= 0):
            continue
        if np.any(depth <= 1e-12):
            i0, i1, k0, k1 = 0, width, 0, height
        else:
            px = corners[:, 0] / depth / (aspect * th)    # in [-1, 1] on screen
            pz = corners[:, 2] / depth / th
            ci = (px + 1) / 2 * width - 0.5
            rj = (1 - pz) / 2 * height - 0.5
            i0 = max(0, int(np.floor(ci.min())) - 1)
            i1 = min(width, int(np.ceil(ci.max())) + 2)
            k0 = max(0, int(np.floor(rj.min())) - 1)
            k1 = min(height, int(np.ceil(rj.max())) + 2)
            if i0 >= i1 or k0 >= k1:
                continue
        dd = D[:, k0:k1, i0:i1]
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (float(r["c"]) - eye[a]) / dd[a]
        p0 = eye[j0] + t * dd[j0]
        p1 = eye[j1] + t * dd[j1]
        ok = ((t > 1e-9) & (p0 >= r["lo"][0]) & (p0 <= r["hi"][0]) &
              (p1 >= r["lo"][1]) & (p1 <= r["hi"][1]) & (t < best_t[k0:k1, i0:i1]))
        best_t[k0:k1, i0:i1][ok] = t[ok]
        best_r[k0:k1, i0:i1][ok] = ri
    best_t = best_t.ravel()
    best_r = best_r.ravel()
    keep = best_r >= 0
    t = best_t[keep]
    r = rects[best_r[keep]]
    pos = eye[:, None] + t[None, :] * D.reshape(3, -1)[:, keep]
    nrm = np.zeros((3, t.size), np.float32)
    for a in range(3):
        m = r["axis"] == a
        pos[a, m] = r["c"][m]          # exactly on the plane
        nrm[a, m] = r["sign"][m]
    pos = np.clip(pos, 0.0, 1.0)
    return np.ascontiguousarray(pos.astype(np.float32)), nrm, best_r[keep]


def hemisphere_dirs(nrm: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Directions uniform over the hemisphere around each (axis-aligned) normal."""
    n = nrm.shape[1]
    v = rng.normal(size=(3, n))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    flip = (v * nrm).sum(0) < 0
    v[:, flip] *= -1
    return np.ascontiguousarray(v.astype(np.float32))


def room_splats(rects: np.ndarray, n: int = 2_000_000, seed: int = 13):
    """Exitance splats: positions uniform by area, outgoing directions uniform
    over the surface normal's hemisphere, RGB i.i.d. LogNormal(0, 1) per channel,
    x100 on emissive rectangles. Returns (pos, wo, rgb), each (3, n) float32."""
    rng = np.random.default_rng(seed)
    pos, nrm, idx = area_points(rects, n, int(rng.integers(1 << 62)))
    wo = hemisphere_dirs(nrm, rng)
    rgb = rng.lognormal(0.0, 1.0, size=(3, n))
    rgb[:, rects["emissive"][idx] != 0] *= 100.0
    return pos, wo, np.ascontiguousarray(rgb.astype(np.float32))


def leaf_splats(leaf_xyz: np.ndarray, leaf_nrm: np.ndarray, leaf_emissive: np.ndarray,
                depth: int, seed: int = 2):
    """One splat per (leaf, side): position at the leaf centre, outgoing
    direction +N for side 0 and -N for side 1, grey RGB = y with y i.i.d.
    LogNormal(0, 1) per leaf-side, x100 on leaves holding an emissive fragment.

    ``leaf_xyz`` is (L, 3) integer leaf coordinates, ``leaf_nrm`` (L, 3) the
    leaf normals, ``leaf_emissive`` (L,) flags. Returns (pos, wo, rgb) SoA with
    2L splats (all side-0 splats first)."""
    rng = np.random.default_rng(seed)
    L = leaf_xyz.shape[0]
    y = rng.lognormal(0.0, 1.0, size=(2, L))
    y[:, leaf_emissive != 0] *= 100.0
    ctr = (leaf_xyz.astype(np.float64) + 0.5) / float(1 << depth)
    pos = np.concatenate([ctr, ctr], 0).T.astype(np.float32)
    wo = np.concatenate([leaf_nrm, -leaf_nrm], 0).T.astype(np.float32)
    rgb = np.repeat(y.reshape(1, -1), 3, 0).astype(np.float32)
    return (np.ascontiguousarray(pos), np.ascontiguousarray(wo), np.ascontiguousarray(rgb))


def bounce_sizes(q0: int, bounces: int = 8, seed: int = 15):
    """Queue sizes q_{i+1} = floor(q_i * s_i), s_i ~ U[0.5, 0.8]."""
    rng = np.random.default_rng(seed)
    q = [int(q0)]
    for _ in range(bounces - 1):
        q.append(int(np.floor(q[-1] * rng.uniform(0.5, 0.8))))
    return q


def bounce_queues(rects: np.ndarray, q0_pos: np.ndarray, q0_nrm: np.ndarray,
                  bounces: int = 8, seed: int = 15):
    """Eight-bounce wavefront: bounce 0 is the given queue, later bounces are
    area-uniform random surface points with decaying sizes."""
    sizes = bounce_sizes(q0_pos.shape[1], bounces, seed)
    out = [(q0_pos, q0_nrm)]
    for b in range(1, bounces):
        p, nn, _ = area_points(rects, sizes[b], seed * 1000 + b)
        out.append((p, nn))
    return out, sizes


def path_wavefront(rects: np.ndarray, P: int, d: int = 8, seed: int = 21, hit_prob: float = 0.7,
                   eye=(0.5, 0.02, 0.5)):
    """Synthetic path memory of a wavefront of P paths of up to d vertices:
    vertex k of every path uniform by area over the rectangles; throughputs
    T_1 ~ U[0.3, 1] per channel, T_k = T_{k-1} * U[0.2, 0.9] (FP32); with
    probability hit_prob a path reaches an emitter at a depth uniform in 1..d
    emitting (12, 11, 9) * U[0.5, 1.5] toward its previous vertex, otherwise
    none (depth -1, zero radiance). Returns (pos (d, 3, P), T (d, 3, P),
    eye (3, P), hit (P,) int32, Le (3, P)), float32 SoA."""
    rng = np.random.default_rng(seed)
    pos = np.empty((d, 3, P), np.float32)
    for k in range(d):
        pos[k] = area_points(rects, P, int(rng.integers(1 << 62)))[0]
    T = np.empty((d, 3, P), np.float32)
    T[0] = rng.uniform(0.3, 1.0, (3, P)).astype(np.float32)
    for k in range(1, d):
        T[k] = T[k - 1] * rng.uniform(0.2, 0.9, (3, P)).astype(np.float32)
    hit = np.where(rng.random(P) < hit_prob, rng.integers(1, d + 1, P), -1).astype(np.int32)
    Le = (np.array([12.0, 11.0, 9.0])[:, None] * rng.uniform(0.5, 1.5, P)[None, :]).astype(np.float32)
    Le[:, hit < 1] = 0.0
    eyes = np.ascontiguousarray(np.tile(np.asarray(eye, np.float32)[:, None], (1, P)))
    return pos, T, eyes, hit, np.ascontiguousarray(Le)
