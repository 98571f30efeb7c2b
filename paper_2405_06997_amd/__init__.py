"""Python binding of libwfpg.so, the MI355X wavefront path-guiding library.

Argument marshalling only: every step of the guiding path runs in the HIP
kernels behind the C ABI declared in ``include/wfpg.h``. PyTorch supplies
device memory (tensors) and the current HIP stream. Device arrays are float32
structure-of-arrays tensors of shape (3, n) (positions, directions, colours)
or (n,) (pdfs). The entry points keep the C names: ``svo_build``,
``svo_accumulate``, ``guide_pdf``, ``guide_sample``, ``pdf_eval``.

Importing this module does not load the library; the first call does, and it
raises ``WfpgLibraryMissing`` if ``libwfpg.so`` has not been built (there is
no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwfpg.so")

WFPG_FP32, WFPG_FP16, WFPG_BF16 = 0, 1, 2
FORMATS = {"fp32": WFPG_FP32, "fp16": WFPG_FP16, "bf16": WFPG_BF16}

STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "device error",
          -4: "invalid state", -5: "unsupported"}

# exported symbols of include/wfpg.h (checked by the CPU test suite)
EXPORTS = [
    "wfpg_default_opts", "wfpg_status_string", "svo_build", "svo_destroy", "svo_accumulate",
    "guide_pdf", "guide_sample", "guide_sample_noalloc", "pdf_eval", "svo_stats", "svo_level_size",
    "svo_export_level",
    "svo_export_accum", "wfpg_dir_table", "wfpg_debug_march", "wfpg_last_error",
    "wfpg_march_counts", "wfpg_get_tile", "wfpg_set_tile", "wfpg_autotune",
    "wfpg_graph_create", "wfpg_graph_launch", "wfpg_graph_destroy", "wfpg_autotune_n",
    "wfpg_default_bin_opts", "wfpg_partition", "guide_sample_binned",
    "guide_sample_product", "pdf_eval_product", "guide_sample_binned_product", "wfpg_dir_table_jitter",
    "svo_accumulate_paths",
    "wfpg_default_train_cfg", "guide_train", "wfpg_nn_param_count", "wfpg_nn_params",
    "wfpg_nn_forward", "wfpg_nn_grad", "wfpg_learned_stats",
]


class WfpgLibraryMissing(ImportError):
    pass


class WfpgError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str = ""):
        msg = f"{fn} failed: {STATUS.get(status, status)} ({status})"
        if detail:
            msg += f" [{detail}]"
        super().__init__(msg)
        self.status = status


class Tile(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32),
                ("blocks_per_cu", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("N", C.c_int32), ("eps", C.c_float), ("mode", C.c_int32),
                ("kl_bound", C.c_float), ("probe_stride", C.c_int32), ("jitter", C.c_int32),
                ("jitter_key", C.c_uint32), ("blur", C.c_int32)]


class BinOpts(C.Structure):
    _fields_ = [("N", C.c_int32), ("eps", C.c_float), ("c_ray", C.c_int32), ("l_min", C.c_int32),
                ("jitter", C.c_int32), ("jitter_key", C.c_uint32), ("blur", C.c_int32)]


class TrainCfg(C.Structure):
    _fields_ = [("log2_table", C.c_int32), ("n_min", C.c_int32), ("n_max", C.c_int32),
                ("batch", C.c_int32), ("steps", C.c_int32), ("lr_mlp", C.c_float),
                ("lr_table", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("adam_eps", C.c_float), ("seed", C.c_uint64), ("target_eps", C.c_float),
                ("target_blur", C.c_int32)]


def make_opts(N: int = 16, eps: float = 0.01, mode: int = 0, kl_bound: float = 0.05,
              probe_stride: int = 256, jitter_key=None, blur: bool = False) -> Opts:
    """Guiding options; jitter_key (not None) turns on the directional jitter
    with that key, blur the Gaussian blur of the field."""
    return Opts(N, eps, mode, kl_bound, probe_stride, int(jitter_key is not None),
                0 if jitter_key is None else jitter_key, int(blur))


_lib = None


def lib():
    """Load libwfpg.so (once) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise WfpgLibraryMissing(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    # torch ships its own HIP runtime under the same SONAME as /opt/rocm's; loading
    # torch first makes the dynamic linker bind this library to that one runtime
    # (two runtimes in one process do not share the device).
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
    sig = {
        "wfpg_default_opts": (Opts, []),
        "wfpg_status_string": (C.c_char_p, [i32]),
        "svo_build": (i32, [vp, i64, i32, i32, vp, C.POINTER(vp)]),
        "svo_destroy": (None, [vp]),
        "svo_accumulate": (i32, [vp, vp, vp, vp, i64, vp]),
        "svo_accumulate_paths": (i32, [vp, vp, vp, vp, vp, vp, i64, i32, vp]),
        "guide_pdf": (i32, [vp, vp, i64, C.POINTER(Opts), vp, vp]),
        "guide_sample": (i32, [vp, vp, vp, i64, u64, u32, C.POINTER(Opts), vp, vp, vp]),
        "guide_sample_noalloc": (i32, [vp, vp, i64, u64, u32, C.POINTER(Opts), vp, vp, vp]),
        "pdf_eval": (i32, [vp, vp, vp, i64, C.POINTER(Opts), vp, vp]),
        "svo_stats": (i32, [vp, vp, vp, vp, vp]),
        "svo_level_size": (i64, [vp, i32]),
        "svo_export_level": (i32, [vp, i32, vp, vp, vp, vp]),
        "svo_export_accum": (i32, [vp, vp, vp, vp]),
        "wfpg_dir_table": (i32, [i32, vp]),
        "wfpg_dir_table_jitter": (i32, [i32, u32, vp]),
        "wfpg_last_error": (C.c_char_p, []),
        "wfpg_march_counts": (i32, [vp, vp, i64, C.POINTER(Opts), vp, vp]),
        "wfpg_get_tile": (i32, [vp, i32, C.POINTER(Tile)]),
        "wfpg_graph_create": (i32, [vp, i32, vp, vp, vp, vp, u64, C.c_float, vp, vp, vp,
                                    C.POINTER(vp)]),
        "wfpg_graph_launch": (i32, [vp, vp]),
        "wfpg_graph_destroy": (None, [vp]),
        "wfpg_set_tile": (i32, [vp, i32, C.POINTER(Tile)]),
        "wfpg_autotune": (i32, [vp, vp, i64, i32, i32, vp, C.POINTER(Tile), C.POINTER(C.c_float)]),
        "wfpg_debug_march": (i32, [vp, vp, i64, C.POINTER(Opts), vp, vp, vp]),
        "wfpg_autotune_n": (i32, [vp, vp, i64, i32, C.c_float, vp, C.POINTER(i32), C.POINTER(Tile),
                                  vp]),
        "wfpg_default_bin_opts": (BinOpts, []),
        "wfpg_partition": (i32, [vp, vp, i64, i32, i32, u64, u32, vp, vp, vp]),
        "guide_sample_binned": (i32, [vp, vp, i64, u64, u32, C.POINTER(BinOpts), vp, vp, vp, vp]),
        "guide_sample_product": (i32, [vp, vp, vp, vp, i64, u64, u32, C.POINTER(Opts), vp, vp, vp]),
        "pdf_eval_product": (i32, [vp, vp, vp, vp, vp, i64, C.POINTER(Opts), vp, vp]),
        "guide_sample_binned_product": (i32, [vp, vp, vp, vp, i64, u64, u32, C.POINTER(BinOpts), vp, vp, vp,
                                              vp]),
        "wfpg_default_train_cfg": (TrainCfg, []),
        "guide_train": (i32, [vp, vp, vp, i64, C.POINTER(TrainCfg), C.POINTER(C.c_float), vp]),
        "wfpg_nn_param_count": (i64, [vp]),
        "wfpg_nn_params": (i32, [vp, vp, i64, i32, vp]),
        "wfpg_nn_forward": (i32, [vp, vp, vp, i64, vp, vp]),
        "wfpg_nn_grad": (i32, [vp, vp, vp, vp, i64, vp, C.POINTER(C.c_float), vp]),
        "wfpg_learned_stats": (i32, [vp, C.POINTER(C.c_float), C.POINTER(i64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(fn: str, st: int):
    if st != 0:
        detail = lib().wfpg_last_error().decode() if st == -3 or st == -2 else ""
        raise WfpgError(fn, st, detail)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t, shape0=None, name="tensor"):
    """Device pointer of a contiguous float32/int32 CUDA tensor."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape0 is not None and (t.dim() != 2 or t.shape[0] != shape0):
        raise ValueError(f"{name} must have shape ({shape0}, n)")
    return C.c_void_p(t.data_ptr())


def dir_table(N: int) -> np.ndarray:
    """FP32 bin-centre directions used by the kernels, (N*N, 3)."""
    out = np.zeros((N * N, 3), np.float32)
    _check("wfpg_dir_table", lib().wfpg_dir_table(N, out.ctypes.data_as(C.c_void_p)))
    return out


def dir_table_jitter(N: int, key: int) -> np.ndarray:
    """FP32 jittered cone directions the kernels use for key, (N*N, 3)."""
    out = np.zeros((N * N, 3), np.float32)
    _check("wfpg_dir_table_jitter", lib().wfpg_dir_table_jitter(N, key, out.ctypes.data_as(C.c_void_p)))
    return out


class SVO:
    """Handle of a device-resident SVO (owns its device memory)."""

    def __init__(self, handle, depth: int, fmt: int):
        self._h = handle
        self.depth = depth
        self.fmt = fmt

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.svo_destroy(self._h)
        self._h = None

    @property
    def handle(self):
        if not self._h:
            raise ValueError("SVO is closed")
        return self._h

    def level_size(self, l: int) -> int:
        return int(lib().svo_level_size(self.handle, l))

    def level_sizes(self):
        return [self.level_size(l) for l in range(self.depth + 1)]

    def stats(self):
        v = [C.c_int64(0), C.c_int64(0), C.c_int64(0)]
        e = C.c_int32(0)
        _check("svo_stats", lib().svo_stats(self.handle, C.byref(v[0]), C.byref(v[1]),
                                            C.byref(v[2]), C.byref(e)))
        return dict(leaves=v[0].value, nodes=v[1].value, dropped=v[2].value, errors=e.value)

    def export_level(self, l: int, stream=None):
        m = self.level_size(l)
        keys = np.zeros(m, np.uint32)
        nrm = np.zeros((m, 3), np.float32)
        ex = np.zeros((m, 2), np.float32)
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        _check("svo_export_level", lib().svo_export_level(self.handle, l, p(keys), p(nrm), p(ex),
                                                          _stream(stream)))
        return keys, nrm, ex

    def export_accum(self, stream=None):
        L = self.level_size(self.depth)
        s = np.zeros((L, 2), np.float32)
        c = np.zeros((L, 2), np.uint32)
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        _check("svo_export_accum", lib().svo_export_accum(self.handle, p(s), p(c), _stream(stream)))
        return s, c


def svo_build(rects: np.ndarray, depth: int, fmt: int = WFPG_FP32, stream=None) -> SVO:
    """Build an SVO from a host array of rectangles (synth.RECT_DTYPE)."""
    r = np.ascontiguousarray(rects)
    if r.dtype.itemsize != 32:
        raise ValueError("rects must use the 32-byte wfpg_rect layout")
    h = C.c_void_p()
    st = lib().svo_build(r.ctypes.data_as(C.c_void_p) if len(r) else None, len(r), depth, fmt,
                         _stream(stream), C.byref(h))
    _check("svo_build", st)
    return SVO(h, depth, fmt)


def svo_accumulate(svo: SVO, pos, wo, rgb, stream=None):
    n = pos.shape[1]
    for t, nm in ((wo, "wo"), (rgb, "rgb")):
        if t.shape != pos.shape:
            raise ValueError(f"{nm} must match pos")
    _check("svo_accumulate", lib().svo_accumulate(svo.handle, _dptr(pos, 3, "pos"), _dptr(wo, 3, "wo"),
                                                  _dptr(rgb, 3, "rgb"), n, _stream(stream)))


def svo_accumulate_paths(svo: SVO, pos, T, eye, hit, Le, stream=None):
    """Eq. 5 extraction: pos, T (d, 3, P), eye, Le (3, P), hit (P,) int32."""
    if pos.dim() != 3 or pos.shape[1] != 3 or T.shape != pos.shape:
        raise ValueError("pos and T must have shape (d, 3, P)")
    d, _, P = pos.shape
    if eye.shape != (3, P) or Le.shape != (3, P) or hit.shape != (P,):
        raise ValueError("eye, Le must be (3, P) and hit (P,)")
    _check("svo_accumulate_paths", lib().svo_accumulate_paths(
        svo.handle, _dptr(pos, name="pos"), _dptr(T, name="T"), _dptr(eye, 3, "eye"), _dptr(hit, name="hit"),
        _dptr(Le, 3, "Le"), P, d, _stream(stream)))


def guide_pdf(svo: SVO, pos, opts: Opts, out=None, stream=None):
    import torch
    n = pos.shape[1]
    NN = opts.N * opts.N
    if out is None:
        out = torch.empty((n, NN), dtype=torch.float32, device=pos.device)
    if out.numel() != n * NN:
        raise ValueError("out must hold n*N*N floats")
    _check("guide_pdf", lib().guide_pdf(svo.handle, _dptr(pos, 3, "pos"), n, C.byref(opts),
                                        _dptr(out, name="out"), _stream(stream)))
    return out


def guide_sample(svo: SVO, pos, opts: Opts, seed: int, bounce: int, nrm=None, dir_out=None,
                 pdf_out=None, stream=None):
    import torch
    n = pos.shape[1]
    if dir_out is None:
        dir_out = torch.empty((3, n), dtype=torch.float32, device=pos.device)
    if pdf_out is None:
        pdf_out = torch.empty((n,), dtype=torch.float32, device=pos.device)
    if dir_out.shape != (3, n) or pdf_out.numel() != n:
        raise ValueError("output shapes must be (3, n) and (n,)")
    _check("guide_sample", lib().guide_sample(
        svo.handle, _dptr(pos, 3, "pos"), _dptr(nrm, 3, "nrm") if nrm is not None else None, n,
        seed, bounce, C.byref(opts), _dptr(dir_out, 3, "dir_out"), _dptr(pdf_out, name="pdf_out"),
        _stream(stream)))
    return dir_out, pdf_out


def guide_sample_noalloc(svo: SVO, pos, opts: Opts, seed: int, bounce: int, dir_out, pdf_out, stream=None):
    """guide_sample into caller-provided outputs (3, n) and (n,) through the
    entry point that allocates no device memory."""
    n = pos.shape[1]
    if dir_out.shape != (3, n) or pdf_out.numel() != n:
        raise ValueError("output shapes must be (3, n) and (n,)")
    _check("guide_sample_noalloc", lib().guide_sample_noalloc(
        svo.handle, _dptr(pos, 3, "pos"), n, seed, bounce, C.byref(opts), _dptr(dir_out, 3, "dir_out"),
        _dptr(pdf_out, name="pdf_out"), _stream(stream)))
    return dir_out, pdf_out


def pdf_eval(svo: SVO, pos, dirs, opts: Opts, out=None, stream=None):
    import torch
    n = pos.shape[1]
    if dirs.shape != pos.shape:
        raise ValueError("dirs must match pos")
    if out is None:
        out = torch.empty((n,), dtype=torch.float32, device=pos.device)
    _check("pdf_eval", lib().pdf_eval(svo.handle, _dptr(pos, 3, "pos"), _dptr(dirs, 3, "dirs"), n,
                                      C.byref(opts), _dptr(out, name="out"), _stream(stream)))
    return out


def _table_ptrs(n, nrm, bsdf):
    """(nrm, bsdf) pointers of a product call: normals (3, n) or tables (n, 64)."""
    if bsdf is not None and bsdf.numel() != 64 * n:
        raise ValueError("bsdf must hold n*64 floats")
    return (_dptr(nrm, 3, "nrm") if nrm is not None else None,
            _dptr(bsdf, name="bsdf") if bsdf is not None else None)


def guide_sample_product(svo: SVO, pos, opts: Opts, seed: int, bounce: int, nrm=None, bsdf=None, dir_out=None,
                         pdf_out=None, stream=None):
    """Product guiding (Sec. 3.6): the vertex field times a BSDF table given
    by normals nrm (3, n; Lambertian) or tables bsdf (n, 64)."""
    import torch
    n = pos.shape[1]
    if dir_out is None:
        dir_out = torch.empty((3, n), dtype=torch.float32, device=pos.device)
    if pdf_out is None:
        pdf_out = torch.empty((n,), dtype=torch.float32, device=pos.device)
    if dir_out.shape != (3, n) or pdf_out.numel() != n:
        raise ValueError("output shapes must be (3, n) and (n,)")
    pn, pb = _table_ptrs(n, nrm, bsdf)
    _check("guide_sample_product", lib().guide_sample_product(
        svo.handle, _dptr(pos, 3, "pos"), pn, pb, n, seed, bounce, C.byref(opts), _dptr(dir_out, 3, "dir_out"),
        _dptr(pdf_out, name="pdf_out"), _stream(stream)))
    return dir_out, pdf_out


def pdf_eval_product(svo: SVO, pos, dirs, opts: Opts, nrm=None, bsdf=None, out=None, stream=None):
    import torch
    n = pos.shape[1]
    if dirs.shape != pos.shape:
        raise ValueError("dirs must match pos")
    if out is None:
        out = torch.empty((n,), dtype=torch.float32, device=pos.device)
    pn, pb = _table_ptrs(n, nrm, bsdf)
    _check("pdf_eval_product", lib().pdf_eval_product(svo.handle, _dptr(pos, 3, "pos"), pn, pb,
                                                      _dptr(dirs, 3, "dirs"), n, C.byref(opts),
                                                      _dptr(out, name="out"), _stream(stream)))
    return out


def debug_march(svo: SVO, pos, opts: Opts, visits: bool = True, stream=None):
    """Test-only traversal records, (n, N*N, 8) int32 and (n, N*N) visits."""
    import torch
    n = pos.shape[1]
    NN = opts.N * opts.N
    out = torch.empty((n, NN, 8), dtype=torch.int32, device=pos.device)
    vis = torch.empty((n, NN), dtype=torch.int32, device=pos.device) if visits else None
    _check("wfpg_debug_march", lib().wfpg_debug_march(
        svo.handle, _dptr(pos, 3, "pos"), n, C.byref(opts), _dptr(out, name="out"),
        _dptr(vis, name="visits") if visits else None, _stream(stream)))
    return out, vis


def march_counts(svo: SVO, pos, opts: Opts, stream=None):
    """Per-vertex (occupancy tests at levels >= 5, hit bins), (n, 2) int32."""
    import torch
    n = pos.shape[1]
    out = torch.empty((n, 2), dtype=torch.int32, device=pos.device)
    _check("wfpg_march_counts", lib().wfpg_march_counts(svo.handle, _dptr(pos, 3, "pos"), n,
                                                        C.byref(opts), _dptr(out, name="counts"),
                                                        _stream(stream)))
    return out


def get_tile(svo: SVO, N: int) -> dict:
    t = Tile()
    _check("wfpg_get_tile", lib().wfpg_get_tile(svo.handle, N, C.byref(t)))
    return dict(waves_per_block=t.waves_per_block, blocks_per_cu=t.blocks_per_cu)


def set_tile(svo: SVO, N: int, waves_per_block: int, blocks_per_cu: int):
    t = Tile(waves_per_block, blocks_per_cu)
    _check("wfpg_set_tile", lib().wfpg_set_tile(svo.handle, N, C.byref(t)))


def autotune(svo: SVO, pos, N: int, reps: int = 3, stream=None) -> dict:
    """Sweep launch shapes on a device queue; caches and returns the best."""
    t = Tile()
    ms = C.c_float(0)
    _check("wfpg_autotune", lib().wfpg_autotune(svo.handle, _dptr(pos, 3, "pos"), pos.shape[1], N,
                                                reps, _stream(stream), C.byref(t), C.byref(ms)))
    return dict(waves_per_block=t.waves_per_block, blocks_per_cu=t.blocks_per_cu, ms=ms.value)


def autotune_n(svo: SVO, pos, budget_ns_per_vertex: float, reps: int = 3, stream=None) -> dict:
    """Finest N in {8, 16, 32} whose tuned time per vertex fits the budget."""
    t = Tile()
    N = C.c_int32(0)
    ms = (C.c_float * 3)()
    _check("wfpg_autotune_n", lib().wfpg_autotune_n(svo.handle, _dptr(pos, 3, "pos"), pos.shape[1], reps,
                                                    budget_ns_per_vertex, _stream(stream), C.byref(N),
                                                    C.byref(t), C.cast(ms, C.c_void_p)))
    return dict(N=N.value, tile=dict(waves_per_block=t.waves_per_block, blocks_per_cu=t.blocks_per_cu),
                ms_per_N={8: ms[0], 16: ms[1], 32: ms[2]})


class BounceGraph:
    """Captured multi-bounce guide_sample (see wfpg_graph_create). Holds
    references to every tensor it was built with."""

    def __init__(self, svo: SVO, queues, n_dev, Ns, seed: int, eps: float = 0.01, stream=None):
        import torch
        self.svo = svo
        self.queues = [q.contiguous() for q in queues]
        self.n_dev = n_dev
        B = len(self.queues)
        cap = [q.shape[1] for q in self.queues]
        self.dirs = [torch.empty((3, c), device=q.device) for c, q in zip(cap, self.queues)]
        self.pdfs = [torch.empty((c,), device=q.device) for c, q in zip(cap, self.queues)]
        P = C.c_void_p * B
        self._pos = P(*[q.data_ptr() for q in self.queues])
        self._dir = P(*[t.data_ptr() for t in self.dirs])
        self._pdf = P(*[t.data_ptr() for t in self.pdfs])
        self._cap = (C.c_int64 * B)(*cap)
        self._N = (C.c_int32 * B)(*Ns)
        if n_dev.dtype != torch.int64 or not n_dev.is_cuda or n_dev.numel() != B:
            raise ValueError("n_dev must be a device int64 tensor with one entry per bounce")
        h = C.c_void_p()
        _check("wfpg_graph_create", lib().wfpg_graph_create(
            svo.handle, B, self._pos, self._cap, C.c_void_p(n_dev.data_ptr()), self._N, seed, eps,
            self._dir, self._pdf, _stream(stream), C.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check("wfpg_graph_launch", lib().wfpg_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.wfpg_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


# ------------------------------------------------------------ learned path

def train_cfg(**kw) -> TrainCfg:
    """Default training configuration with fields overridden by keyword."""
    c = lib().wfpg_default_train_cfg()
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def guide_train(svo: SVO, pos, nrm, cfg: TrainCfg | None = None, stream=None, **kw) -> float:
    """Adam steps of the learned model on march targets; returns the mean loss
    of the last steps."""
    n = pos.shape[1]
    if nrm.shape != pos.shape:
        raise ValueError("nrm must match pos")
    cfg = cfg if cfg is not None else train_cfg(**kw)
    loss = C.c_float(0)
    _check("guide_train", lib().guide_train(svo.handle, _dptr(pos, 3, "pos"), _dptr(nrm, 3, "nrm"),
                                            n, C.byref(cfg), C.byref(loss), _stream(stream)))
    return float(loss.value)


def nn_param_count(svo: SVO) -> int:
    return int(lib().wfpg_nn_param_count(svo.handle))


def nn_get_params(svo: SVO, stream=None) -> np.ndarray:
    n = nn_param_count(svo)
    if n < 0:
        raise WfpgError("wfpg_nn_params", -4)
    out = np.zeros(n, np.float32)
    _check("wfpg_nn_params", lib().wfpg_nn_params(svo.handle, out.ctypes.data_as(C.c_void_p), n, 0,
                                                  _stream(stream)))
    return out


def nn_set_params(svo: SVO, params: np.ndarray, stream=None):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check("wfpg_nn_params", lib().wfpg_nn_params(svo.handle, p.ctypes.data_as(C.c_void_p), p.size, 1,
                                                  _stream(stream)))


def nn_forward(svo: SVO, pos, nrm, out=None, stream=None):
    import torch
    n = pos.shape[1]
    if out is None:
        out = torch.empty((n, 256), dtype=torch.float32, device=pos.device)
    if out.numel() != n * 256:
        raise ValueError("out must hold n*256 floats")
    _check("wfpg_nn_forward", lib().wfpg_nn_forward(svo.handle, _dptr(pos, 3, "pos"),
                                                    _dptr(nrm, 3, "nrm"), n, _dptr(out, name="out"),
                                                    _stream(stream)))
    return out


def nn_grad(svo: SVO, pos, nrm, target, stream=None):
    """(loss, gradient tensor) of the mean cross-entropy against target (n, 256)."""
    import torch
    n = pos.shape[1]
    if target.shape != (n, 256):
        raise ValueError("target must be (n, 256)")
    g = torch.empty((nn_param_count(svo),), dtype=torch.float32, device=pos.device)
    loss = C.c_float(0)
    _check("wfpg_nn_grad", lib().wfpg_nn_grad(svo.handle, _dptr(pos, 3, "pos"), _dptr(nrm, 3, "nrm"),
                                              _dptr(target, name="target"), n, _dptr(g, name="grad"),
                                              C.byref(loss), _stream(stream)))
    return float(loss.value), g


def learned_stats(svo: SVO) -> dict:
    kl = C.c_float(0)
    fb = C.c_int64(0)
    _check("wfpg_learned_stats", lib().wfpg_learned_stats(svo.handle, C.byref(kl), C.byref(fb)))
    return {"last_probe_kl": float(kl.value), "fallbacks": int(fb.value)}


# ------------------------------------------------------ positional binning

def bin_opts(N: int = 16, eps: float = 0.01, c_ray: int = 512, l_min: int = 5, jitter_key=None,
             blur: bool = False) -> BinOpts:
    return BinOpts(N, eps, c_ray, l_min, int(jitter_key is not None), 0 if jitter_key is None else jitter_key,
                   int(blur))


def partition(svo: SVO, pos, c_ray: int, l_min: int, seed: int = 0, bounce: int = 0, stream=None):
    """(bin global node index, origin queue index) per query, int32 tensors."""
    import torch
    n = pos.shape[1]
    b = torch.empty((n,), dtype=torch.int32, device=pos.device)
    o = torch.empty((n,), dtype=torch.int32, device=pos.device)
    _check("wfpg_partition", lib().wfpg_partition(svo.handle, _dptr(pos, 3, "pos"), n, c_ray, l_min, seed,
                                                  bounce, _dptr(b, name="bin"), _dptr(o, name="origin"),
                                                  _stream(stream)))
    return b, o


def guide_sample_binned(svo: SVO, pos, opts: BinOpts, seed: int, bounce: int, dir_out=None, pdf_out=None,
                        bins: bool = False, stream=None):
    """Per-bin fields sampled by every member: (dir (3, n), pdf (n,)[, bin (n,)])."""
    import torch
    n = pos.shape[1]
    if dir_out is None:
        dir_out = torch.empty((3, n), dtype=torch.float32, device=pos.device)
    if pdf_out is None:
        pdf_out = torch.empty((n,), dtype=torch.float32, device=pos.device)
    b = torch.empty((n,), dtype=torch.int32, device=pos.device) if bins else None
    _check("guide_sample_binned", lib().guide_sample_binned(
        svo.handle, _dptr(pos, 3, "pos"), n, seed, bounce, C.byref(opts), _dptr(dir_out, 3, "dir_out"),
        _dptr(pdf_out, name="pdf_out"), _dptr(b, name="bin") if bins else None, _stream(stream)))
    return (dir_out, pdf_out, b) if bins else (dir_out, pdf_out)


def guide_sample_binned_product(svo: SVO, pos, opts: BinOpts, seed: int, bounce: int, nrm=None, bsdf=None,
                                dir_out=None, pdf_out=None, bins: bool = False, stream=None):
    """Binned product guiding: every member's table times its bin's field."""
    import torch
    n = pos.shape[1]
    if dir_out is None:
        dir_out = torch.empty((3, n), dtype=torch.float32, device=pos.device)
    if pdf_out is None:
        pdf_out = torch.empty((n,), dtype=torch.float32, device=pos.device)
    b = torch.empty((n,), dtype=torch.int32, device=pos.device) if bins else None
    pn, pb = _table_ptrs(n, nrm, bsdf)
    _check("guide_sample_binned_product", lib().guide_sample_binned_product(
        svo.handle, _dptr(pos, 3, "pos"), pn, pb, n, seed, bounce, C.byref(opts), _dptr(dir_out, 3, "dir_out"),
        _dptr(pdf_out, name="pdf_out"), _dptr(b, name="bin") if bins else None, _stream(stream)))
    return (dir_out, pdf_out, b) if bins else (dir_out, pdf_out)
