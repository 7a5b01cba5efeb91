"""The C-ABI library loads on this host and exports every function that
include/lightfuse.h declares (no compute calls: no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lightfuse.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2608_29269_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("liblightfuse.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2608_29269_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_params_default_values(lib):
    from paper_2608_29269_amd import _lib
    p = _lib.Params()
    lib.lf_params_default(C.byref(p))
    assert (p.k, p.spp, p.seed, p.flags) == (32, 1, 0, 0)
    assert p.alpha_min == 1.0 / 255.0 and p.alpha_cap == 0.99 and p.support_sigma == 3.0
    assert p.eps == 1e-6 and p.t_min == 1e-4 and p.secondary_offset == 1e-3


def test_null_context_paths(lib):
    assert lib.lf_last_error(None) == b"null context"
    assert lib.lf_sync(None) == 1
    assert lib.lf_scene_refit(None) == 1
    assert lib.lf_create(None, 0, None) == 1


def test_struct_sizes_match_header(lib):
    from paper_2608_29269_amd import _lib
    assert C.sizeof(_lib.Camera) == 12 * 4 + 4 + 4 + 4
    assert C.sizeof(_lib.Params) == 4 + 4 + 8 + 6 * 8 + 8  # trailing uint32 padded to 8
    assert C.sizeof(_lib.Surfels) == 7 * 8 + 8 + 8 + 8
