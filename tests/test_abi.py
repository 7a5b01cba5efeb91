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
    assert lib.lf_abort(None) == 1
    assert lib.lf_sync_timeout(None, C.c_double(1.0)) == 1


def test_struct_sizes_match_header(lib):
    from paper_2608_29269_amd import _lib
    assert C.sizeof(_lib.Camera) == 12 * 4 + 4 + 4 + 4
    assert C.sizeof(_lib.Params) == 4 + 4 + 8 + 6 * 8 + 8  # trailing uint32 padded to 8
    assert C.sizeof(_lib.Surfels) == 7 * 8 + 8 + 8 + 8


def _c_layout(tmp_path):
    """sizeof and field offsets of every ABI struct, as a C compiler sees the header."""
    import subprocess
    from paper_2608_29269_amd import _lib
    structs = {"lf_surfels": _lib.Surfels, "lf_transforms": _lib.Transforms, "lf_envmap": _lib.EnvMap,
               "lf_rays": _lib.Rays, "lf_camera": _lib.Camera, "lf_params": _lib.Params, "lf_outputs": _lib.Outputs,
               "lf_grad_out": _lib.GradOut, "lf_grad_in": _lib.GradIn, "lf_scene_info": _lib.SceneInfo,
               "lf_render_stats": _lib.RenderStats, "lf_server_config": _lib.ServerConfig,
               "lf_request": _lib.Request, "lf_server_stats": _lib.ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {}
    for ln in out:
        if ln:
            cname, key, val = ln.split()
            got[(cname, key)] = int(val)
    return structs, got


def test_ctypes_layout_matches_the_c_compiler(tmp_path):
    structs, got = _c_layout(tmp_path)
    for cname, py in structs.items():
        assert C.sizeof(py) == got[(cname, "size")], cname
        for f, _ in py._fields_:
            assert getattr(py, f).offset == got[(cname, f)], (cname, f)


def test_server_null_paths_and_defaults(lib):
    from paper_2608_29269_amd import _lib
    assert lib.lf_server_last_error(None) == b"null server"
    assert lib.lf_server_create(None, None, None) == 1
    assert lib.lf_server_submit(None, None, None) == 1
    assert lib.lf_server_poll(None, 1, None) == 1
    lib.lf_server_destroy(None)
    cfg = _lib.ServerConfig()
    lib.lf_server_config_default(C.byref(cfg))
    assert (cfg.max_slots, cfg.tile_rays, cfg.batch_rays, cfg.max_spp) == (16, 65536, 1048576, 4)
    assert cfg.hbm_budget_bytes == 16 << 30 and cfg.tile_rays % 128 == 0 and cfg.batch_rays % 128 == 0
    assert cfg.params.k == 32 and cfg.params.alpha_min == 1.0 / 255.0
    assert cfg.policy == _lib.SCHED_OLDEST_FIRST and cfg.max_in_flight == 2


def test_binding_constants_match_the_header():
    from paper_2608_29269_amd import _lib
    src = open(HEADER).read()
    assert int(re.search(r"#define LF_NUM_COUNTERS (\d+)", src).group(1)) == _lib.NUM_COUNTERS
    for name in ("NO_SECONDARY", "NO_BACKGROUND", "BSDF_ONLY", "DIFFUSE_ONLY", "BRUTE_FORCE", "COUNT", "UNSORTED",
                 "NEE", "SOBOL", "DETERMINISTIC"):
        m = re.search(r"#define LF_FLAG_%s\s+\(1u << (\d+)\)" % name, src)
        assert m and getattr(_lib, "FLAG_" + name) == 1 << int(m.group(1)), name


def test_status_codes_match_the_header():
    from paper_2608_29269_amd import _lib
    src = open(HEADER).read()
    codes = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"\b(LF_[A-Z]+) = (\d+)", src))
    assert codes["LF_OK"] == 0 and len(codes) == len(_lib.STATUS_NAMES)
    for name, v in codes.items():
        assert getattr(_lib, name) == v and _lib.STATUS_NAMES[v] == name, name


def compile_c_demo(tmp_path):
    """Builds tests/c_abi_demo.c with gcc against the header, the built
    library and the HIP runtime (C API only)."""
    import subprocess
    from paper_2608_29269_amd import _lib
    lib_dir = os.path.dirname(_lib.LIB_PATH)
    exe = tmp_path / "c_abi_demo"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "c_abi_demo.c"), "-L" + lib_dir, "-llightfuse",
                           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath," + lib_dir, "-Wl,-rpath,/opt/rocm/lib", "-lm",
                           "-o", str(exe)])
    return exe


def test_c_caller_compiles_and_links(lib, tmp_path):
    """A plain C99 program that drives the whole boundary (scene, render,
    backward, errors) compiles warning-free against the header and links
    against the library (it runs in the GPU tests)."""
    assert compile_c_demo(tmp_path).exists()

