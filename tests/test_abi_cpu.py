"""The C-ABI library loads, exports every symbol include/rcp.h declares, and
rejects invalid arguments on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import scenegen
from paper_2312_12392_amd import rcp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "rcp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rcp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_names():
    assert header_functions() == sorted(rcp.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(rcp.LIB_PATH):
        pytest.skip("librcp.so not built")
    L = ctypes.CDLL(rcp.LIB_PATH)
    for name in header_functions():
        assert hasattr(L, name), name


def test_status_strings():
    rcp.load()
    assert rcp.status_string(rcp.RCP_OK) == "ok"
    assert rcp.status_string(rcp.RCP_ERR_INVALID_ARGUMENT) == "invalid argument"
    assert rcp.status_string(99) == "unknown status"


def _bad(fn, *a, **k):
    with pytest.raises(rcp.RcpError) as e:
        fn(*a, **k)
    assert e.value.status == rcp.RCP_ERR_INVALID_ARGUMENT
    return str(e.value)


def test_render_argument_validation_on_host():
    cam = scenegen.workload("soup256").camera
    d = rcp.make_displacement(0.0, 0.02)
    assert "scene is NULL" in _bad(rcp.rcp_render, 0, cam, 64, 64, 6, d, 1, None, stream=0)
    # camera and displacement checks run before any device call
    bad_cam = scenegen.Camera(eye=[0, 0, 0], right=[2, 0, 0], up=[0, 1, 0], forward=[0, 0, 1], tan_half_fovy=0.5)
    assert "unit" in _bad(rcp.rcp_generate_rays, bad_cam, 8, 8, d, None, 1, 1, stream=0)
    skew = scenegen.Camera(eye=[0, 0, 0], right=[1, 0, 0], up=[0.6, 0.8, 0], forward=[0, 0, 1], tan_half_fovy=0.5)
    assert "orthogonal" in _bad(rcp.rcp_generate_rays, skew, 8, 8, d, None, 1, 1, stream=0)
    nan_cam = scenegen.Camera(eye=[np.nan, 0, 0], right=[1, 0, 0], up=[0, 1, 0], forward=[0, 0, 1], tan_half_fovy=0.5)
    _bad(rcp.rcp_generate_rays, nan_cam, 8, 8, d, None, 1, 1, stream=0)
    for le, ld in [(-0.1, 0.0), (0.0, 1.0), (0.0, -0.01), (np.inf, 0.0)]:
        _bad(rcp.rcp_generate_rays, cam, 8, 8, rcp.make_displacement(le, ld), None, 1, 1, stream=0)
    _bad(rcp.rcp_generate_rays, cam, 8, 8, rcp.make_displacement(0.0, 0.1, mode=7), None, 1, 1, stream=0)
    for W, H in [(0, 8), (8, 0), (-1, 5), (1 << 14, (1 << 13) + 1)]:
        _bad(rcp.rcp_generate_rays, cam, W, H, d, None, 1, 1, stream=0)
    _bad(rcp.rcp_generate_rays, cam, 8, 8, d, None, None, 1, stream=0)
    _bad(rcp.rcp_render_stats, 0, cam, 8, 8, 1, d, 1, None, stream=0)


def test_build_argument_validation_on_host():
    sc = scenegen.soup_scene(0, 16)
    bad = scenegen.Scene(verts=sc.verts, idx=sc.idx.copy(), rgb=sc.rgb)
    bad.idx[3, 1] = sc.n_verts
    assert "out of range" in _bad(rcp.rcp_build_scene, bad, stream=0)
    nanv = scenegen.Scene(verts=sc.verts.copy(), idx=sc.idx, rgb=sc.rgb)
    nanv.verts[5, 2] = np.nan
    assert "not finite" in _bad(rcp.rcp_build_scene, nanv, stream=0)
    nanc = scenegen.Scene(verts=sc.verts, idx=sc.idx, rgb=sc.rgb.copy())
    nanc.rgb[0, 0] = np.inf
    _bad(rcp.rcp_build_scene, nanc, stream=0)
    nbg = scenegen.Scene(verts=sc.verts, idx=sc.idx, rgb=sc.rgb, background=[np.nan, 0, 0])
    _bad(rcp.rcp_build_scene, nbg, stream=0)
    for opts in [rcp.build_options(max_leaf=0), rcp.build_options(max_leaf=9), rcp.build_options(c_trav=-1.0),
                 rcp.build_options(c_trav=0.0), rcp.build_options(c_isect=np.nan), rcp.build_options(builder=2),
                 rcp.build_options(builder=-1), rcp.build_options(collapse=2), rcp.build_options(collapse=-1)]:
        _bad(rcp.rcp_build_scene, sc, opts, stream=0)


def test_trace_and_sort_validation_on_host():
    _bad(rcp.rcp_trace_rays, 0, 1, 1, 4, 1, 1, stream=0)
    _bad(rcp.rcp_radix_sort_u64, 1, 1, -1, stream=0)
    _bad(rcp.rcp_radix_sort_u64, None, None, 5, stream=0)
    rcp.rcp_radix_sort_u64(None, None, 0, stream=0)   # empty is a no-op
    with pytest.raises(rcp.RcpError):
        rcp.rcp_scene_info(0)


def test_last_error_is_cleared_by_a_successful_call():
    rcp.load()
    with pytest.raises(rcp.RcpError):
        rcp.rcp_scene_info(0)
    assert rcp.last_error() != ""
    rcp.rcp_radix_sort_u64(None, None, 0, stream=0)
    assert rcp.last_error() == ""


def test_binding_requires_the_built_library(tmp_path):
    import importlib
    mod = importlib.import_module("paper_2312_12392_amd.rcp")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(RuntimeError, match="missing"):
            mod.load(str(tmp_path / "nope.so"))
    finally:
        mod._lib = saved


def test_gather_validation_on_host():
    _bad(rcp.rcp_gather_passes, None, 8, 8, 1, 2.0, rcp.RCP_EDGE_MIRROR, True, 1 << 20, stream=0)
    _bad(rcp.rcp_gather_passes, 1 << 20, 8, 8, 0, 2.0, rcp.RCP_EDGE_MIRROR, True, 1 << 30, stream=0)
    _bad(rcp.rcp_gather_passes, 1 << 20, 8, 8, 65, 2.0, rcp.RCP_EDGE_MIRROR, True, 1 << 30, stream=0)
    _bad(rcp.rcp_gather_passes, 1 << 20, 8, 8, 1, -1.0, rcp.RCP_EDGE_MIRROR, True, 1 << 30, stream=0)
    _bad(rcp.rcp_gather_passes, 1 << 20, 8, 8, 1, float("nan"), rcp.RCP_EDGE_MIRROR, True, 1 << 30, stream=0)
    _bad(rcp.rcp_gather_passes, 1 << 20, 8, 8, 1, 2.0, 3, True, 1 << 30, stream=0)
    _bad(rcp.rcp_gather_passes, 1 << 20, 0, 8, 1, 2.0, rcp.RCP_EDGE_WRAP, True, 1 << 30, stream=0)
    # the output planes must not overlap the input image
    assert "overlaps" in _bad(rcp.rcp_gather_passes, 1 << 20, 8, 8, 2, 2.0, rcp.RCP_EDGE_WRAP, True,
                              (1 << 20) + 100, stream=0)


def test_server_validation_on_host():
    _bad(rcp.rcp_server_create, 0, 1 << 20)
    cam = scenegen.workload("soup256").camera
    with pytest.raises(rcp.RcpError):
        rcp.rcp_submit(0, cam, 8, 8, 2, rcp.make_displacement(0.0, 0.02))
    with pytest.raises(rcp.RcpError):
        rcp.rcp_poll(0, 1)
    with pytest.raises(rcp.RcpError):
        rcp.rcp_release(0, 1)


def test_header_constants_match_the_binding():
    import re
    text = open(HEADER).read() if "HEADER" in globals() else open(
        os.path.join(os.path.dirname(__file__), "..", "include", "rcp.h")).read()
    defs = dict(re.findall(r"#define\s+(RCP_[A-Z_]+)\s+(-?\d+)", text))
    assert defs, "no integer constants found in the header"
    for name, value in defs.items():
        assert hasattr(rcp, name), f"binding lacks {name}"
        assert getattr(rcp, name) == int(value), name
