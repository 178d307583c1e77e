"""Host-side checks of the C ABI library (no GPU needed): it loads and exports
every function include/pstereo.h declares, and the binding's parameter struct
matches the header's layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pstereo.h")


def _declared():
    src = open(os.path.join(ROOT, "include", "pstereo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pstereo_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2009_09501_amd.pstereo import LIB_PATH, load_library
    if not os.path.exists(LIB_PATH):
        from paper_2009_09501_amd.build import build_library
        build_library()
    return load_library()


def test_header_declares_core_calls():
    d = _declared()
    for name in ("pstereo_create", "pstereo_synthesize", "pstereo_destroy"):
        assert name in d


def test_library_exports_every_declared_symbol(lib):
    from paper_2009_09501_amd.pstereo import EXPORTED
    declared = _declared()
    assert sorted(EXPORTED) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_params_struct_layout(lib):
    from paper_2009_09501_amd.pstereo import PstereoParams
    p = PstereoParams()
    assert lib.pstereo_params_init(ctypes.byref(p)) == 0
    assert p.struct_size == ctypes.sizeof(PstereoParams)
    assert (p.max_disparity, p.depth_threshold, p.block_size, p.edge_thresh,
            p.link_thresh, p.cbf_radius, p.flags) == (-1, 150, 0, 24, 24, 2, 0)


def test_null_and_bad_args_without_gpu(lib):
    """Argument checks that return before touching a device."""
    assert lib.pstereo_params_init(None) == -1
    assert lib.pstereo_synthesize(None, None, 1, 1, None, None, None, None) == -1
    assert lib.pstereo_destroy(None) == 0
    h = ctypes.c_void_p()
    assert lib.pstereo_create(ctypes.byref(h), 0, 0, 10) == -1
    assert b"out of range" in lib.pstereo_last_error(None)


def test_completion_struct_layout():
    """pstereo_completion: u64 id, i32 stream, i32 status, three doubles."""
    from paper_2009_09501_amd.pstereo import PstereoCompletion
    assert ctypes.sizeof(PstereoCompletion) == 40
    assert [PstereoCompletion.__dict__[f].offset for f in
            ("req_id", "stream_id", "status", "t_submit", "t_launch", "t_done")] == [0, 8, 12, 16, 24, 32]


def test_batch_tuning_struct_layout():
    """pstereo_batch_tuning: the header's int32 fields in order (mode,
    warp_lanes, warp_rows, fused_grid, bs_rows) and the trial record after
    it (tuning, then a double)."""
    from paper_2009_09501_amd.pstereo import PstereoBatchTrial, PstereoBatchTuning
    hdr = open(HEADER).read()
    body = re.search(r"typedef struct pstereo_batch_tuning \{(.*?)\} pstereo_batch_tuning;", hdr, re.S).group(1)
    fields = re.findall(r"int32_t\s+(\w+);", body)
    assert [f for f, _ in PstereoBatchTuning._fields_] == fields
    assert ctypes.sizeof(PstereoBatchTuning) == 4 * len(fields)
    assert PstereoBatchTrial.ms.offset == (4 * len(fields) + 7) // 8 * 8


def test_header_constants_match_binding():
    """Every flag, error code and mode the header #defines has the same value
    in the Python binding."""
    import paper_2009_09501_amd.pstereo as ps
    defs = re.findall(r"#define (PSTEREO_[A-Z0-9_]+) \(?(-?(?:0x[0-9a-fA-F]+|\d+))u?\)?", open(HEADER).read())
    assert len(defs) >= 20
    for name, val in defs:
        if name == "PSTEREO_NOALLOC_MAX_PIXELS":
            continue
        assert getattr(ps, name) == int(val, 0), name


def test_server_bad_args_without_gpu(lib):
    s = ctypes.c_void_p()
    assert lib.pstereo_server_create(0, 0, 8, 2, 0, ctypes.byref(s)) == -1      # no budget
    assert lib.pstereo_server_create(0, 1 << 30, 0, 2, 0, ctypes.byref(s)) == -1  # no streams
    assert lib.pstereo_server_create(0, 1 << 30, 8, 0, 0, ctypes.byref(s)) == -1  # no lanes
    assert lib.pstereo_server_create(0, 1 << 30, 8, 2, 7, ctypes.byref(s)) == -1  # unknown policy
    assert lib.pstereo_server_submit(None, 0, None, None, None, None, None) == -1
    assert lib.pstereo_server_destroy(None) == 0


@pytest.mark.parametrize("lang,compiler", [("c", "gcc"), ("c++", "g++")])
def test_header_compiles_standalone(lang, compiler, tmp_path):
    """The public header is self-contained C (and C++): a translation unit
    that includes only it compiles without warnings."""
    import shutil
    import subprocess
    if not shutil.which(compiler):
        pytest.skip(f"{compiler} not available")
    src = tmp_path / ("use.c" if lang == "c" else "use.cc")
    src.write_text('#include "pstereo.h"\nint main(void) { pstereo_params p; return pstereo_params_init(&p); }\n')
    r = subprocess.run([compiler, "-fsyntax-only", "-Wall", "-Wextra", "-Werror", "-I", os.path.dirname(HEADER),
                        str(src)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
