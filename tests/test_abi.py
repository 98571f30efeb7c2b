"""CPU checks of the C ABI: the library loads, exports every function that
include/wfpg.h declares, and its host-side direction table matches the
oracle's bit for bit. No device work is issued."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "wfpg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_matches_binding_exports():
    import paper_2405_06997_amd as w
    assert sorted(w.EXPORTS) == declared_functions()


def test_library_exports_all_symbols():
    import paper_2405_06997_amd as w
    lib = w.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_defaults():
    import paper_2405_06997_amd as w
    lib = w.lib()
    assert lib.wfpg_status_string(0) == b"ok"
    assert lib.wfpg_status_string(-1) == b"invalid argument"
    o = lib.wfpg_default_opts()
    assert (o.N, o.mode, o.probe_stride) == (16, 0, 256)
    assert abs(o.eps - 0.01) < 1e-9 and abs(o.kl_bound - 0.05) < 1e-9
    assert (o.jitter, o.jitter_key, o.blur) == (0, 0, 0)
    b = lib.wfpg_default_bin_opts()
    assert (b.N, b.c_ray, b.l_min, b.jitter, b.blur) == (16, 512, 5, 0, 0)


@pytest.mark.parametrize("N", [8, 16, 32])
def test_dir_table_bitexact_vs_oracle(orc, N):
    import paper_2405_06997_amd as w
    got = w.dir_table(N)
    want = orc.dir_table(N)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_invalid_arguments_rejected_without_device():
    """Validation happens before any device work (NULL handles, bad N)."""
    import paper_2405_06997_amd as w
    lib = w.lib()
    o = w.make_opts(N=12)
    assert lib.guide_pdf(None, None, 0, C.byref(o), None, None) == -1
    assert lib.svo_accumulate(None, None, None, None, 0, None) == -1
    h = C.c_void_p()
    assert lib.svo_build(None, 0, 11, 0, None, C.byref(h)) == -1
    assert lib.svo_build(None, 0, 6, 7, None, C.byref(h)) == -1
    o16 = w.make_opts(N=16)
    assert lib.guide_sample_product(None, None, None, None, 0, 0, 0, C.byref(o16), None, None, None) == -1
    assert lib.pdf_eval_product(None, None, None, None, None, 0, C.byref(o16), None, None) == -1
    bo = w.bin_opts()
    assert lib.guide_sample_binned_product(None, None, None, None, 0, 0, 0, C.byref(bo), None, None, None,
                                           None) == -1
    assert lib.svo_accumulate_paths(None, None, None, None, None, None, 0, 4, None) == -1
    assert lib.wfpg_dir_table_jitter(12, 0, None) == -1
    assert lib.wfpg_dir_table(12, None) == -1
    assert lib.svo_level_size(None, 0) == -1
