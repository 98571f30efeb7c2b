"""CPU oracle for the wavefront path-guiding hot path (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never calls it and shares no code with it.
The arithmetic lives in ``oracle.c`` (plain C, FP64 values, exact integer
traversal, FP32 only where an integer decision is taken in the paper's FP32);
this module only marshals numpy arrays through ctypes.

Parity unpinned: none of the functions below. Every function is pinned by a
test in ``tests/test_oracle_*.py`` against closed forms, brute force or
invariants that do not reuse this code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC_NN = os.path.join(_HERE, "nn_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FMT_FP32, FMT_FP16, FMT_BF16 = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP contraction off)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
            _SRC, _SRC_NN, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        vp, i32, i64, u32, u64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float
        sig = {
            "orc_build": (vp, [vp, i64, i32, vp]),
            "orc_free": (None, [vp]),
            "orc_depth": (i32, [vp]),
            "orc_level_size": (i64, [vp, i32]),
            "orc_level_keys": (None, [vp, i32, vp]),
            "orc_level_normals": (None, [vp, i32, vp]),
            "orc_level_exitance": (None, [vp, i32, vp, vp]),
            "orc_leaf_info": (None, [vp, vp, vp]),
            "orc_leaf_accum": (None, [vp, vp, vp, vp]),
            "orc_dropped": (i64, [vp]),
            "orc_set_uniform_exitance": (None, [vp, f32]),
            "orc_accumulate": (i64, [vp, vp, vp, vp, i64]),
            "orc_propagate": (None, [vp, i32]),
            "orc_morton": (u32, [u32, u32, u32]),
            "orc_oct_decode": (None, [C.c_double, C.c_double, vp]),
            "orc_oct_encode": (None, [C.c_double, C.c_double, C.c_double, vp]),
            "orc_dir_table": (None, [i32, vp]),
            "orc_philox": (None, [vp, vp, vp]),
            "orc_debug_march": (None, [vp, vp, i64, i32, i32, i32, vp, vp]),
            "orc_field": (None, [vp, vp, i64, i32, f32, vp, vp]),
            "orc_guide_pdf": (None, [vp, vp, i64, i32, f32, vp, vp]),
            "orc_guide_sample": (None, [vp, vp, i64, u64, u32, i32, f32, vp, vp, vp, vp, vp]),
            "orc_pdf_eval": (None, [vp, vp, vp, i64, i32, f32, vp, vp, vp]),
            "orc_partition": (None, [vp, vp, i64, i32, i32, vp, vp]),
            "orc_binned_sample": (None, [vp, vp, i64, i32, i32, u64, u32, i32, f32, vp, vp, vp, vp, vp, vp,
                                         vp, vp, vp, i32, u32, i32]),
            "orc_jitter_table": (None, [i32, u32, vp]),
            "orc_path_splats": (i64, [vp, vp, vp, vp, vp, i64, i32, vp, vp, vp, i64]),
            "orc_blur": (None, [vp, i32, vp]),
            "orc_field_aa": (None, [vp, vp, i64, i32, f32, i32, u32, i32, vp]),
            "orc_sample_fields": (None, [vp, i64, i64, i32, u64, u32, vp, vp, vp, vp, vp]),
            "orc_product_fields": (None, [vp, i64, i64, i32, vp, vp, u64, u32, vp, vp, vp, vp, vp]),
            "orc_product_pdf_fields": (None, [vp, i64, i32, vp, vp, vp, vp]),
            "orc_product_sample": (None, [vp, vp, vp, vp, i64, u64, u32, i32, f32, vp, vp, vp, vp]),
            "orc_product_pdf_eval": (None, [vp, vp, vp, vp, vp, i64, i32, f32, vp, vp, vp]),
            "orc_march_one": (None, [vp, vp, vp, i32, i32, vp]),
            "orc_quantize": (None, [vp, vp, vp, vp]),
            "orc_round_fmt_array": (None, [vp, vp, i64, i32]),
            "orc_eval_one": (None, [vp, vp, vp, i32, vp, vp]),
            "orc_oct_encode_many": (None, [vp, i64, vp]),
            "orc_oct_decode_many": (None, [vp, i64, vp]),
            "orc_num_threads": (i32, []),
            "orc_set_num_threads": (None, [i32]),
            "orc_nn_mlp_params": (i64, []),
            "orc_nn_num_params": (i64, [vp]),
            "orc_nn_resolutions": (None, [vp, vp]),
            "orc_nn_forward": (None, [vp, vp, vp, vp, i64, i32, vp, vp]),
            "orc_nn_grad": (C.c_double, [vp, vp, vp, vp, vp, i64, i32, vp]),
            "orc_nn_inputs": (None, [vp, vp, vp, vp, i64, i32, vp]),
            "orc_nn_parity_bounds": (None, [vp, vp, vp, vp, vp, i64, C.c_double, vp, vp]),
            "orc_kl_rows": (None, [vp, vp, i64, vp]),
            "orc_nn_encode_info": (None, [vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _soa(a, dtype=np.float32):
    a = np.ascontiguousarray(a, dtype=dtype)
    assert a.ndim == 2 and a.shape[0] == 3
    return a


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int):
    lib().orc_set_num_threads(t)


def morton(x: int, y: int, z: int) -> int:
    return int(lib().orc_morton(x, y, z))


def oct_decode(x: float, y: float) -> np.ndarray:
    out = np.zeros(3)
    lib().orc_oct_decode(x, y, _p(out))
    return out


def oct_encode(d) -> np.ndarray:
    out = np.zeros(2)
    lib().orc_oct_encode(float(d[0]), float(d[1]), float(d[2]), _p(out))
    return out


def oct_encode_many(d) -> np.ndarray:
    """(3, n) directions -> (2, n) square coordinates."""
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros((2, d.shape[1]))
    lib().orc_oct_encode_many(_p(d), d.shape[1], _p(out))
    return out


def oct_decode_many(xy) -> np.ndarray:
    """(2, n) square coordinates -> (3, n) unit directions."""
    xy = np.ascontiguousarray(xy, np.float64)
    out = np.zeros((3, xy.shape[1]))
    lib().orc_oct_decode_many(_p(xy), xy.shape[1], _p(out))
    return out


def dir_table(N: int) -> np.ndarray:
    """(N*N, 3) float32 bin-centre directions, bin b = v*N + u."""
    out = np.zeros((N * N, 3), np.float32)
    lib().orc_dir_table(N, _p(out))
    return out


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox(_p(c), _p(k), _p(o))
    return o


def round_fmt(x, fmt: int) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32).ravel()
    out = np.empty_like(x)
    lib().orc_round_fmt_array(_p(x), _p(out), x.size, fmt)
    return out


def quantize(p, d):
    p = np.ascontiguousarray(p, np.float32)
    d = np.ascontiguousarray(d, np.float32)
    O = np.zeros(3, np.int64)
    q = np.zeros(3, np.int64)
    lib().orc_quantize(_p(p), _p(d), _p(O), _p(q))
    return O, q


class SVO:
    """Oracle sparse voxel octree built from axis-aligned rectangles."""

    def __init__(self, rects: np.ndarray, depth: int):
        self._rects = np.ascontiguousarray(rects)
        assert self._rects.dtype.itemsize == 32
        st = C.c_int32(0)
        h = lib().orc_build(_p(self._rects), len(self._rects), depth, C.byref(st))
        if not h:
            raise ValueError(f"orc_build failed with status {st.value}")
        self._h = h
        self.depth = depth

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def level_size(self, l: int) -> int:
        return int(lib().orc_level_size(self._h, l))

    def level_sizes(self):
        return [self.level_size(l) for l in range(self.depth + 1)]

    def keys(self, l: int) -> np.ndarray:
        out = np.zeros(self.level_size(l), np.uint32)
        lib().orc_level_keys(self._h, l, _p(out))
        return out

    def normals(self, l: int) -> np.ndarray:
        out = np.zeros((self.level_size(l), 3), np.float32)
        lib().orc_level_normals(self._h, l, _p(out))
        return out

    def exitance(self, l: int):
        n = self.level_size(l)
        e32 = np.zeros((n, 2), np.float32)
        e64 = np.zeros((n, 2), np.float64)
        lib().orc_level_exitance(self._h, l, _p(e32), _p(e64))
        return e32, e64

    def leaf_info(self):
        L = self.level_size(self.depth)
        xyz = np.zeros((L, 3), np.int32)
        em = np.zeros(L, np.uint8)
        lib().orc_leaf_info(self._h, _p(xyz), _p(em))
        return xyz, em

    def leaf_accum(self):
        L = self.level_size(self.depth)
        s32 = np.zeros((L, 2), np.float32)
        s64 = np.zeros((L, 2), np.float64)
        cnt = np.zeros((L, 2), np.int64)
        lib().orc_leaf_accum(self._h, _p(s32), _p(s64), _p(cnt))
        return s32, s64, cnt

    def dropped(self) -> int:
        return int(lib().orc_dropped(self._h))

    def set_uniform_exitance(self, v: float):
        lib().orc_set_uniform_exitance(self._h, v)

    def accumulate(self, pos, wo, rgb) -> int:
        pos, wo, rgb = _soa(pos), _soa(wo), _soa(rgb)
        return int(lib().orc_accumulate(self._h, _p(pos), _p(wo), _p(rgb), pos.shape[1]))

    def propagate(self, fmt: int = FMT_FP32):
        lib().orc_propagate(self._h, fmt)

    def march_one(self, p, d, hier=False, lds_levels=5):
        p = np.ascontiguousarray(p, np.float32)
        d = np.ascontiguousarray(d, np.float32)
        out = np.zeros(5, np.int64)
        lib().orc_march_one(self._h, _p(p), _p(d), int(hier), lds_levels, _p(out))
        return dict(hit=int(out[0]), axis=int(out[1]), key=int(out[2]), delta=int(out[3]),
                    visits=int(out[4]))

    def eval_one(self, p, d, N: int):
        p = np.ascontiguousarray(p, np.float32)
        d = np.ascontiguousarray(d, np.float32)
        out = np.zeros(8, np.int64)
        val = np.zeros(2)
        lib().orc_eval_one(self._h, _p(p), _p(d), N, _p(out), _p(val))
        keys = ("hit", "axis", "leaf", "delta", "k", "node", "node_index", "side")
        rec = {k: int(v) for k, v in zip(keys, out)}
        rec["value"], rec["r"] = float(val[0]), float(val[1])
        return rec

    def debug_march(self, pos, N: int, lds_levels: int = 5, hier: bool = False,
                    visits: bool = False):
        """(n, N*N, 8) int64 records {hit, axis, leaf, delta, k, node, node_index,
        side} and optionally (n, N*N) node-test counts."""
        pos = _soa(pos)
        n = pos.shape[1]
        out = np.zeros((n, N * N, 8), np.int64)
        vis = np.zeros((n, N * N), np.int64) if visits else None
        lib().orc_debug_march(self._h, _p(pos), n, N, lds_levels, int(hier), _p(out),
                              _p(vis) if visits else None)
        return (out, vis) if visits else out

    def field(self, pos, N: int, eps: float = 0.01):
        pos = _soa(pos)
        n = pos.shape[1]
        L = np.zeros((n, N * N))
        Lt = np.zeros((n, N * N))
        lib().orc_field(self._h, _p(pos), n, N, eps, _p(L), _p(Lt))
        return L, Lt

    def guide_pdf(self, pos, N: int, eps: float = 0.01, truth: bool = False):
        pos = _soa(pos)
        n = pos.shape[1]
        pdf = np.zeros((n, N * N))
        pt = np.zeros((n, N * N)) if truth else None
        lib().orc_guide_pdf(self._h, _p(pos), n, N, eps, _p(pdf), _p(pt) if truth else None)
        return (pdf, pt) if truth else pdf

    def guide_sample(self, pos, N: int, seed: int, bounce: int, eps: float = 0.01, counter=None):
        """counter: RNG counter per vertex (its index in the full queue);
        defaults to 0..n-1."""
        pos = _soa(pos)
        n = pos.shape[1]
        ctr = None if counter is None else np.ascontiguousarray(counter, np.int64)
        d = np.zeros((3, n))
        pdf = np.zeros(n)
        b = np.zeros((n, 2), np.int32)
        m = np.zeros((n, 2))
        lib().orc_guide_sample(self._h, _p(pos), n, seed, bounce, N, eps,
                               _p(ctr) if ctr is not None else None, _p(d), _p(pdf), _p(b), _p(m))
        return dict(dir=d, pdf=pdf, bin=b, margin=m)

    def partition(self, pos, c_ray: int, l_min: int):
        """Positional bins (Alg. 2): (level, index within level) per query."""
        pos = _soa(pos)
        n = pos.shape[1]
        lv = np.zeros(n, np.int32)
        ix = np.zeros(n, np.int64)
        lib().orc_partition(self._h, _p(pos), n, c_ray, l_min, _p(lv), _p(ix))
        return lv, ix

    def binned_sample(self, pos, c_ray: int, l_min: int, N: int, seed: int, bounce: int,
                      eps: float = 0.01, nrm=None, bsdf=None, jitter_key=None, blur: bool = False):
        """Per-bin fields and member samples (Alg. 2 + Alg. 3); with nrm or
        bsdf every member draws a product sample (Sec. 3.6) instead;
        jitter_key / blur: the field antialiasing of field_aa."""
        pos = _soa(pos)
        n = pos.shape[1]
        nv, bv = _product_inputs(nrm, bsdf, n)
        d = np.zeros((3, n))
        pdf = np.zeros(n)
        b = np.zeros((n, 2), np.int32)
        m = np.zeros((n, 2))
        lv = np.zeros(n, np.int32)
        ix = np.zeros(n, np.int64)
        org = np.zeros(n, np.int64)
        lib().orc_binned_sample(self._h, _p(pos), n, c_ray, l_min, seed, bounce, N, eps, _p(d), _p(pdf),
                                _p(b), _p(m), _p(lv), _p(ix), _p(org), _opt(nv), _opt(bv),
                                int(jitter_key is not None), 0 if jitter_key is None else jitter_key, int(blur))
        return dict(dir=d, pdf=pdf, bin=b, margin=m, level=lv, index=ix, origin=org)

    def field_aa(self, pos, N: int, jitter_key=None, blur: bool = False, eps: float = 0.01):
        """Fields (n x N*N) with directional jitter (jitter_key not None)
        and/or the Gaussian blur (Sec. 4)."""
        pos = _soa(pos)
        n = pos.shape[1]
        L = np.zeros((n, N * N))
        lib().orc_field_aa(self._h, _p(pos), n, N, eps, int(jitter_key is not None),
                           0 if jitter_key is None else jitter_key, int(blur), _p(L))
        return L

    def product_sample(self, pos, N: int, seed: int, bounce: int, nrm=None, bsdf=None, eps: float = 0.01):
        """Product guiding (Sec. 3.6) of each vertex's own field; nrm (3 x n,
        Lambertian cosine table) or bsdf (n x 64 table)."""
        pos = _soa(pos)
        n = pos.shape[1]
        nv, bv = _product_inputs(nrm, bsdf, n, need=True)
        d = np.zeros((3, n))
        pdf = np.zeros(n)
        b = np.zeros((n, 2), np.int32)
        m = np.zeros((n, 2))
        lib().orc_product_sample(self._h, _p(pos), _opt(nv), _opt(bv), n, seed, bounce, N, eps, _p(d), _p(pdf),
                                 _p(b), _p(m))
        return dict(dir=d, pdf=pdf, bin=b, margin=m)

    def product_pdf_eval(self, pos, dirs, N: int, nrm=None, bsdf=None, eps: float = 0.01):
        pos = _soa(pos)
        dirs = _soa(dirs)
        n = pos.shape[1]
        nv, bv = _product_inputs(nrm, bsdf, n, need=True)
        pdf = np.zeros(n)
        b = np.zeros((n, 2), np.int32)
        e = np.zeros(n)
        lib().orc_product_pdf_eval(self._h, _p(pos), _opt(nv), _opt(bv), _p(dirs), n, N, eps, _p(pdf), _p(b),
                                   _p(e))
        return dict(pdf=pdf, bin=b, edge=e)

    def pdf_eval(self, pos, dirs, N: int, eps: float = 0.01):
        pos = _soa(pos)
        dirs = _soa(dirs)
        n = pos.shape[1]
        pdf = np.zeros(n)
        b = np.zeros((n, 2), np.int32)
        e = np.zeros(n)
        lib().orc_pdf_eval(self._h, _p(pos), _p(dirs), n, N, eps, _p(pdf), _p(b), _p(e))
        return dict(pdf=pdf, bin=b, edge=e)


def _opt(a):
    return None if a is None else _p(a)


def _product_inputs(nrm, bsdf, n, need=False):
    if nrm is not None and bsdf is not None:
        raise ValueError("give nrm or bsdf, not both")
    if need and nrm is None and bsdf is None:
        raise ValueError("product guiding needs nrm or bsdf")
    nv = None if nrm is None else _soa(nrm)
    bv = None if bsdf is None else np.ascontiguousarray(bsdf, np.float32).reshape(n, 64)
    assert nv is None or nv.shape[1] == n
    return nv, bv


def product_sample_fields(L, N: int, seed: int, bounce: int, nrm=None, bsdf=None, counter=None, n=None):
    """Product sample (Sec. 3.6) from given fields L (n x N*N, rows v); a
    single row with n given is one field shared by n queries."""
    L = np.ascontiguousarray(L, np.float64).reshape(-1, N * N)
    shared = n is not None and L.shape[0] == 1
    n = L.shape[0] if n is None else n
    assert (shared or L.shape[0] == n) and N % 8 == 0
    nv, bv = _product_inputs(nrm, bsdf, n, need=True)
    ctr = None if counter is None else np.ascontiguousarray(counter, np.int64)
    d = np.zeros((3, n))
    pdf = np.zeros(n)
    b = np.zeros((n, 2), np.int32)
    m = np.zeros((n, 2))
    lib().orc_product_fields(_p(L), 0 if shared else N * N, n, N, _opt(nv), _opt(bv), seed, bounce, _opt(ctr),
                             _p(d), _p(pdf), _p(b), _p(m))
    return dict(dir=d, pdf=pdf, bin=b, margin=m)


def path_splats(pos, T, eye, hit, Le):
    """Eq. 5 splats of a wavefront: pos, T (d, 3, P), eye, Le (3, P), hit (P,)
    -> (spos, swo, srgb) each 3 x m, depth-major."""
    pos = np.ascontiguousarray(pos, np.float32)
    T = np.ascontiguousarray(T, np.float32)
    d, _, P = pos.shape
    eye = _soa(eye)
    Le = _soa(Le)
    hit = np.ascontiguousarray(hit, np.int32)
    cap = max(1, d * P)
    sp = np.zeros((3, cap), np.float32)
    sw = np.zeros((3, cap), np.float32)
    sr = np.zeros((3, cap), np.float32)
    m = lib().orc_path_splats(_p(pos), _p(T), _p(eye), _p(hit), _p(Le), P, d, _p(sp), _p(sw), _p(sr), cap)
    assert m >= 0
    return (np.ascontiguousarray(sp[:, :m]), np.ascontiguousarray(sw[:, :m]), np.ascontiguousarray(sr[:, :m]))


def jitter_table(N: int, key: int) -> np.ndarray:
    """FP32 jittered cone directions (N*N, 3) for jitter key `key`."""
    out = np.zeros((N * N, 3), np.float32)
    lib().orc_jitter_table(N, key, _p(out))
    return out


def blur(L, N: int) -> np.ndarray:
    """The 3 x 3 binomial blur of fields L (... x N*N) with edge folding."""
    L = np.ascontiguousarray(L, np.float64)
    flat = L.reshape(-1, N * N)
    out = np.zeros_like(flat)
    for k in range(flat.shape[0]):
        lib().orc_blur(_p(flat[k]), N, _p(out[k]))
    return out.reshape(L.shape)


def sample_fields(L, N: int, seed: int, bounce: int, counter=None, n=None):
    """guide_sample's rule on given fields (n x N*N; one shared row with n)."""
    L = np.ascontiguousarray(L, np.float64).reshape(-1, N * N)
    shared = n is not None and L.shape[0] == 1
    n = L.shape[0] if n is None else n
    ctr = None if counter is None else np.ascontiguousarray(counter, np.int64)
    d = np.zeros((3, n))
    pdf = np.zeros(n)
    b = np.zeros((n, 2), np.int32)
    m = np.zeros((n, 2))
    lib().orc_sample_fields(_p(L), 0 if shared else N * N, n, N, seed, bounce, _opt(ctr), _p(d), _p(pdf), _p(b),
                            _p(m))
    return dict(dir=d, pdf=pdf, bin=b, margin=m)


def product_pdf_fields(L, N: int, dirs, nrm=None, bsdf=None):
    """Product pdf of directions (3 x n) under fields L (n x N*N)."""
    L = np.ascontiguousarray(L, np.float64)
    n = L.shape[0]
    nv, bv = _product_inputs(nrm, bsdf, n, need=True)
    d = np.ascontiguousarray(dirs, np.float64)
    pdf = np.zeros(n)
    lib().orc_product_pdf_fields(_p(L), n, N, _opt(nv), _opt(bv), _p(d), _p(pdf))
    return pdf


# ---------------------------------------------------------------- learned --
class NNCfg(C.Structure):
    _fields_ = [("log2_table", C.c_int32), ("n_min", C.c_int32), ("n_max", C.c_int32)]


NN_LEVELS, NN_FEAT, NN_IN, NN_H, NN_OUT = 16, 2, 35, 64, 256


def nn_cfg(log2_table: int = 19, n_min: int = 16, n_max: int = 1024) -> NNCfg:
    return NNCfg(log2_table, n_min, n_max)


def nn_num_params(cfg: NNCfg) -> int:
    return int(lib().orc_nn_num_params(C.byref(cfg)))


def nn_mlp_params() -> int:
    return int(lib().orc_nn_mlp_params())


def nn_resolutions(cfg: NNCfg) -> np.ndarray:
    out = np.zeros(NN_LEVELS, np.int32)
    lib().orc_nn_resolutions(C.byref(cfg), _p(out))
    return out


def nn_forward(params, cfg: NNCfg, pos, nrm, mode: int = 0):
    """(probabilities, logits), each (n, 256) FP64. mode 1 = BF16-faithful."""
    params = np.ascontiguousarray(params, np.float32)
    pos, nrm = _soa(pos), _soa(nrm)
    n = pos.shape[1]
    prob = np.zeros((n, NN_OUT))
    logit = np.zeros((n, NN_OUT))
    lib().orc_nn_forward(_p(params), C.byref(cfg), _p(pos), _p(nrm), n, mode, _p(prob), _p(logit))
    return prob, logit


def nn_grad(params, cfg: NNCfg, pos, nrm, target, mode: int = 0):
    """(loss, gradient over all parameters) of the mean cross-entropy."""
    params = np.ascontiguousarray(params, np.float32)
    pos, nrm = _soa(pos), _soa(nrm)
    target = np.ascontiguousarray(target, np.float64)
    g = np.zeros(nn_num_params(cfg))
    loss = lib().orc_nn_grad(_p(params), C.byref(cfg), _p(pos), _p(nrm), _p(target),
                             pos.shape[1], mode, _p(g))
    return float(loss), g


def nn_parity_bounds(params, cfg: NNCfg, pos, nrm, target=None, inv_b: float = 1.0):
    """Bounds of the GPU's arithmetic against the BF16-faithful mode (see
    orc_nn_parity_bounds): the relative bound of every probability (n, 256)
    and, with a target, the radius around the mode-1 gradient (batch scale
    inv_b) that each gradient element must lie within."""
    params = np.ascontiguousarray(params, np.float32)
    pos, nrm = _soa(pos), _soa(nrm)
    n = pos.shape[1]
    pe = np.zeros((n, 256))
    t = None if target is None else np.ascontiguousarray(target, np.float64)
    gr = np.zeros(nn_num_params(cfg)) if t is not None else None
    lib().orc_nn_parity_bounds(_p(params), C.byref(cfg), _p(pos), _p(nrm), None if t is None else _p(t), n,
                               float(inv_b), _p(pe), None if gr is None else _p(gr))
    return pe, gr


def nn_inputs(params, cfg: NNCfg, pos, nrm, mode: int = 1):
    """The network's input rows (n x 35): encoded features, then the normal."""
    params = np.ascontiguousarray(params, np.float32)
    pos, nrm = _soa(pos), _soa(nrm)
    x = np.zeros((pos.shape[1], 35))
    lib().orc_nn_inputs(_p(params), C.byref(cfg), _p(pos), _p(nrm), pos.shape[1], mode, _p(x))
    return x


def kl_rows(p, q) -> np.ndarray:
    p = np.ascontiguousarray(p, np.float64)
    q = np.ascontiguousarray(q, np.float64)
    out = np.zeros(p.shape[0])
    lib().orc_kl_rows(_p(p), _p(q), p.shape[0], _p(out))
    return out


def nn_encode_info(cfg: NNCfg, p):
    p = np.ascontiguousarray(p, np.float32)
    idx = np.zeros((NN_LEVELS, 8), np.uint32)
    w = np.zeros((NN_LEVELS, 8))
    lib().orc_nn_encode_info(C.byref(cfg), _p(p), _p(idx), _p(w))
    return idx, w
