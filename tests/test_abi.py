"""C-ABI checks that need no GPU: the library loads, exports every function
include/gscache.h declares, and rejects bad arguments with error codes
(no compute call is made)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gscache.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsc_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_2502_14938_amd as gs
    return gs.lib()


def test_header_declares_the_frame_calls():
    fns = declared_functions()
    for name in ("gsc_load_anchors", "gsc_set_camera_pair", "gsc_derive", "gsc_render_stereo",
                 "gsc_render_gaussians", "gsc_create", "gsc_destroy", "gsc_last_error"):
        assert name in fns
    assert len(fns) >= 25


def test_library_exports_every_declared_symbol(L):
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    import paper_2502_14938_amd as gs
    assert set(declared_functions()) == set(gs.SYMBOLS)


def test_null_and_invalid_arguments(L):
    import paper_2502_14938_amd as gs
    h = C.c_void_p()
    assert L.gsc_create(None, None, C.byref(h)) == -1
    assert b"null" in L.gsc_last_error(None)
    cfg = gs.Config()
    cfg.k, cfg.feat_dim, cfg.hidden, cfg.d_max = 10, 32, 32, 10
    cfg.max_width, cfg.max_height = 64, 64
    bad = gs.Config.from_buffer_copy(cfg); bad.k = 0
    assert L.gsc_create(C.byref(bad), None, C.byref(h)) == -1
    bad = gs.Config.from_buffer_copy(cfg); bad.feat_dim = 16
    assert L.gsc_create(C.byref(bad), None, C.byref(h)) == -1
    bad = gs.Config.from_buffer_copy(cfg); bad.d_max = 64
    assert L.gsc_create(C.byref(bad), None, C.byref(h)) == -1
    bad = gs.Config.from_buffer_copy(cfg); bad.precision = 7
    assert L.gsc_create(C.byref(bad), None, C.byref(h)) == -1
    bad = gs.Config.from_buffer_copy(cfg); bad.max_width = 0
    assert L.gsc_create(C.byref(bad), None, C.byref(h)) == -1
    # calls on a null context fail cleanly
    assert L.gsc_derive(None) == -1
    assert L.gsc_sync(None) == -1
    assert L.gsc_render_stereo(None, None, None, None, None) == -1
    assert L.gsc_set_camera_pair(None, None, None, 0.0) == -1
    n = C.c_int64()
    assert L.gsc_debug_copy(None, 0, 0, None, 0, C.byref(n)) == -1
    assert L.gsc_pipeline(None, 1) == -1
    assert L.gsc_timing_stages(None, 1) == -1
    assert L.gsc_count_work(None, 1) == -1
    assert L.gsc_server_policy(None, 0.0, 0.0, 0.0, 0) == -1
    out = C.c_double()
    assert L.gsc_ssim(None, None, None, 3, 16, 16, C.byref(out)) == -1
    L.gsc_destroy(None)


def test_struct_sizes_match_header():
    import subprocess
    import tempfile
    import paper_2502_14938_amd as gs
    code = ('#include <stdio.h>\n#include "gscache.h"\nint main(void){printf("%zu %zu %zu %zu %zu %zu",'
            'sizeof(gsc_config),sizeof(gsc_camera),sizeof(gsc_anchors),sizeof(gsc_mlp),sizeof(gsc_gaussians),'
            'sizeof(gsc_frame_stats));return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "s.c"), os.path.join(d, "s")
        open(src, "w").write(code)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        got = list(map(int, subprocess.check_output([exe]).split()))
    want = [C.sizeof(x) for x in (gs.Config, gs.Camera, gs.Anchors, gs.Mlp, gs.Gaussians, gs.FrameStats)]
    assert got == want


def test_noalloc_entry_rejects_sizes_beyond_its_maxima(L):
    """The allocation-free entry checks its arguments before any device work
    (so these run without a GPU); its maxima match the header's."""
    import paper_2502_14938_amd as gs
    src = open(HEADER).read()
    for name, val in (("GSC_NOALLOC_MAX_GAUSSIANS", gs.NOALLOC_MAX_GAUSSIANS),
                      ("GSC_NOALLOC_MAX_PAIRS", gs.NOALLOC_MAX_PAIRS), ("GSC_NOALLOC_MAX_SIDE", gs.NOALLOC_MAX_SIDE)):
        m = re.search(r"#define %s \(?([0-9]+)(?: << ([0-9]+))?\)?" % name, src)
        assert m, name
        assert (int(m.group(1)) << int(m.group(2) or 0)) == val, name
    assert L.gsc_render_gaussians_noalloc(None, None, None, None, None, None) == -1
    g = gs.Gaussians()
    g.n = gs.NOALLOC_MAX_GAUSSIANS + 1
    g.mu = g.cov = g.rgb = g.alpha = 16  # never dereferenced: the size check comes first
    cam = gs.camera({"R": [1, 0, 0, 0, 1, 0, 0, 0, 1], "pos": [0, 0, 0], "fovx": 1.0, "fovy": 1.0, "width": 64,
                     "height": 64, "znear": 0.2})
    out = C.c_void_p(16)
    assert L.gsc_render_gaussians_noalloc(C.byref(g), C.byref(cam), out, None, None, None) == -1
    assert b"GSC_NOALLOC_MAX_GAUSSIANS" in L.gsc_last_error(None)
    g.n = -1
    assert L.gsc_render_gaussians_noalloc(C.byref(g), C.byref(cam), out, None, None, None) == -1
    g.n = 10
    cam.width = gs.NOALLOC_MAX_SIDE + 1
    assert L.gsc_render_gaussians_noalloc(C.byref(g), C.byref(cam), out, None, None, None) == -1
    assert b"GSC_NOALLOC_MAX_SIDE" in L.gsc_last_error(None)
