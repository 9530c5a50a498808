"""ctypes binding of librcp.so (the C ABI in include/rcp.h).

Argument marshalling only: every step of the render runs in the library's
HIP kernels.  Device buffers are passed as torch CUDA tensors (or raw device
addresses as ints); streams as torch streams, raw hipStream_t ints, or None
for torch's current stream.  Functions keep the C names; each raises
``RcpError`` when the call returns a status other than RCP_OK.

There is no fallback: if librcp.so has not been built, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librcp.so")

RCP_OK = 0
RCP_ERR_INVALID_ARGUMENT = 1
RCP_ERR_OUT_OF_MEMORY = 2
RCP_ERR_DEVICE = 3
RCP_ERR_NOT_READY = 4
RCP_ERR_QUEUE_FULL = 5
RCP_ERR_INTERNAL = 6
RCP_MODE_COLOR = 0
RCP_MODE_DEPTH = 1
RCP_MODE_NORMAL = 2
RCP_BUILDER_PLOC = 0
RCP_BUILDER_LBVH = 1
RCP_COLLAPSE_SAH = 0
RCP_COLLAPSE_GREEDY = 1
RCP_ENGINE_CHAIN = 0
RCP_ENGINE_PASSES = 1
ENGINE_CHAIN, ENGINE_PASSES = RCP_ENGINE_CHAIN, RCP_ENGINE_PASSES
RCP_EDGE_CLAMP = 0
RCP_EDGE_WRAP = 1
RCP_EDGE_MIRROR = 2
RCP_REQ_QUEUED, RCP_REQ_RUNNING, RCP_REQ_DONE, RCP_REQ_FAILED = 0, 1, 2, 3

# Every symbol include/rcp.h declares.
EXPORTED = [
    "rcp_build_scene", "rcp_destroy_scene", "rcp_scene_info", "rcp_render", "rcp_render_pass",
    "rcp_render_stats", "rcp_generate_rays", "rcp_trace_rays", "rcp_export_bvh", "rcp_radix_sort_u64",
    "rcp_status_string", "rcp_last_error", "rcp_gather_passes", "rcp_render_batch", "rcp_graph_create",
    "rcp_graph_update", "rcp_graph_launch", "rcp_graph_destroy", "rcp_get_tuning", "rcp_set_tuning", "rcp_autotune",
    "rcp_server_create", "rcp_submit", "rcp_poll", "rcp_result", "rcp_result_copy", "rcp_release", "rcp_server_stats",
    "rcp_server_destroy", "rcp_check", "rcp_debug_set", "rcp_render_noalloc", "rcp_render_noalloc_scratch_bytes",
    "rcp_autotune_batch",
]
STAT_COLS = 6
RCP_DEBUG_FAIL_ALLOC_AFTER = 1
RCP_DEBUG_STEP_BUDGET = 2
RCP_DEBUG_LIST_CANARY = 3


class RcpError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: status {status} ({status_string(status)}): {msg}")
        self.status = status


class rcp_scene_desc(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("n_verts", ctypes.c_uint32), ("idx", ctypes.c_void_p),
                ("n_tris", ctypes.c_uint32), ("tri_rgb", ctypes.c_void_p), ("light_dir", ctypes.c_float * 3),
                ("k_a", ctypes.c_float), ("k_d", ctypes.c_float), ("background", ctypes.c_float * 3)]


class rcp_camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("right", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("forward", ctypes.c_float * 3), ("tan_half_fovy", ctypes.c_float)]


class rcp_displacement(ctypes.Structure):
    _fields_ = [("lambda_eye", ctypes.c_float), ("lambda_dir", ctypes.c_float), ("mode", ctypes.c_int32),
                ("z0", ctypes.c_float)]


class rcp_build_options(ctypes.Structure):
    _fields_ = [("max_leaf", ctypes.c_int32), ("c_trav", ctypes.c_float),
                ("c_isect", ctypes.c_float), ("builder", ctypes.c_int32), ("collapse", ctypes.c_int32)]


class rcp_view(ctypes.Structure):
    _fields_ = [("camera", rcp_camera), ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("K", ctypes.c_int32),
                ("disp", rcp_displacement), ("out_images", ctypes.c_void_p), ("out_ids", ctypes.c_void_p)]


class rcp_tuning(ctypes.Structure):
    _fields_ = [("refill_min", ctypes.c_int32), ("exit_lanes", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("tile_log2w", ctypes.c_int32), ("engine", ctypes.c_int32), ("top_levels", ctypes.c_int32),
                ("stack_entries", ctypes.c_int32), ("block_size", ctypes.c_int32), ("tile_order", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class rcp_request(ctypes.Structure):
    _fields_ = [("camera", rcp_camera), ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("K", ctypes.c_int32),
                ("disp", rcp_displacement), ("with_ids", ctypes.c_int32)]


class rcp_scene_stats(ctypes.Structure):
    _fields_ = [("n_tris", ctypes.c_uint32), ("n_nodes", ctypes.c_uint32), ("n_leaves", ctypes.c_uint32),
                ("max_depth", ctypes.c_uint32), ("max_leaf", ctypes.c_uint32),
                ("sah_cost", ctypes.c_float), ("build_ms", ctypes.c_float), ("device_bytes", ctypes.c_uint64),
                ("node_bytes", ctypes.c_uint32), ("leaf_hist", ctypes.c_uint32 * 8)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["leaf_hist"] = list(self.leaf_hist)
        return d


_lib = None


def load(path: str | None = None):
    """Load librcp.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build the HIP library first (python __graft_entry__.py build)")
    # torch ships its own HIP runtime (libamdhip64.so.7).  Loading torch first
    # makes librcp.so bind to that same runtime instead of pulling a second
    # copy from /opt/rocm into the process, so device pointers and streams
    # from torch are valid in the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(p)
    P = ctypes.c_void_p
    i32 = ctypes.c_int
    st = ctypes.c_int
    sig = {
        "rcp_build_scene": (st, [ctypes.POINTER(rcp_scene_desc), ctypes.POINTER(rcp_build_options), P,
                                 ctypes.POINTER(P)]),
        "rcp_destroy_scene": (None, [P]),
        "rcp_scene_info": (st, [P, ctypes.POINTER(rcp_scene_stats)]),
        "rcp_render": (st, [P, ctypes.POINTER(rcp_camera), i32, i32, i32, ctypes.POINTER(rcp_displacement), P, P, P]),
        "rcp_render_pass": (st, [P, ctypes.POINTER(rcp_camera), i32, i32, ctypes.POINTER(rcp_displacement), P, P, P,
                                 P, P, P]),
        "rcp_render_stats": (st, [P, ctypes.POINTER(rcp_camera), i32, i32, i32, ctypes.POINTER(rcp_displacement), P,
                                  P, P, P]),
        "rcp_generate_rays": (st, [ctypes.POINTER(rcp_camera), i32, i32, ctypes.POINTER(rcp_displacement), P, P, P,
                                   P, P]),
        "rcp_trace_rays": (st, [P, P, P, i32, P, P, P, P]),
        "rcp_export_bvh": (st, [P, P, P]),
        "rcp_radix_sort_u64": (st, [P, P, i32, P]),
        "rcp_gather_passes": (st, [P, i32, i32, i32, ctypes.c_float, i32, i32, P, P]),
        "rcp_server_create": (st, [P, ctypes.c_uint64, i32, i32, ctypes.POINTER(P)]),
        "rcp_submit": (st, [P, ctypes.POINTER(rcp_request), ctypes.POINTER(ctypes.c_uint64)]),
        "rcp_poll": (st, [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), P]),
        "rcp_result": (st, [P, ctypes.c_uint64, ctypes.POINTER(P), ctypes.POINTER(P)]),
        "rcp_result_copy": (st, [P, ctypes.c_uint64, P, P, P]),
        "rcp_release": (st, [P, ctypes.c_uint64]),
        "rcp_server_stats": (st, [P, P]),
        "rcp_server_destroy": (None, [P]),
        "rcp_render_batch": (st, [P, ctypes.POINTER(rcp_view), i32, P]),
        "rcp_graph_create": (st, [P, ctypes.POINTER(rcp_camera), i32, i32, i32, ctypes.POINTER(rcp_displacement), P, P,
                                  P, ctypes.POINTER(P)]),
        "rcp_graph_update": (st, [P, ctypes.POINTER(rcp_camera), ctypes.POINTER(rcp_displacement)]),
        "rcp_graph_launch": (st, [P, P]),
        "rcp_graph_destroy": (None, [P]),
        "rcp_get_tuning": (st, [P, ctypes.POINTER(rcp_tuning)]),
        "rcp_set_tuning": (st, [P, ctypes.POINTER(rcp_tuning)]),
        "rcp_autotune": (st, [P, ctypes.POINTER(rcp_camera), i32, i32, i32, ctypes.POINTER(rcp_displacement), P, P, i32,
                              ctypes.POINTER(rcp_tuning), ctypes.POINTER(ctypes.c_float), P]),
        "rcp_render_noalloc": (st, [P, ctypes.POINTER(rcp_camera), i32, i32, i32, ctypes.POINTER(rcp_displacement),
                                    P, P, P]),
        "rcp_render_noalloc_scratch_bytes": (ctypes.c_uint64, []),
        "rcp_check": (st, [P, P]),
        "rcp_debug_set": (st, [i32, ctypes.c_int64]),
        "rcp_autotune_batch": (st, [P, ctypes.POINTER(rcp_view), i32, i32, ctypes.POINTER(rcp_tuning),
                                    ctypes.POINTER(ctypes.c_float), P]),
        "rcp_status_string": (ctypes.c_char_p, [st]),
        "rcp_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_string(s: int) -> str:
    return load().rcp_status_string(int(s)).decode()


def last_error() -> str:
    return load().rcp_last_error().decode()


def _check(status: int, func: str):
    if status != RCP_OK:
        raise RcpError(status, func, last_error())


def _dev_ptr(t):
    """Device address of a torch tensor (or an int address); None -> NULL."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("expected a device (CUDA/HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _f3(v):
    return [float(x) for x in np.asarray(v, dtype=np.float32).reshape(3)]


def make_camera(cam) -> rcp_camera:
    """From any object with eye/right/up/forward/tan_half_fovy."""
    c = rcp_camera()
    c.eye[:] = _f3(cam.eye)
    c.right[:] = _f3(cam.right)
    c.up[:] = _f3(cam.up)
    c.forward[:] = _f3(cam.forward)
    c.tan_half_fovy = float(np.float32(cam.tan_half_fovy))
    return c


def make_displacement(lambda_eye: float, lambda_dir: float, mode: int = RCP_MODE_COLOR,
                      z0: float = 0.0) -> rcp_displacement:
    d = rcp_displacement()
    d.lambda_eye = float(lambda_eye)
    d.lambda_dir = float(lambda_dir)
    d.mode = int(mode)
    d.z0 = float(z0)
    return d


# ---------------------------------------------------------------------------
# The C entry points, one to one
# ---------------------------------------------------------------------------

def rcp_build_scene(scene, opts: rcp_build_options | None = None, stream=None) -> int:
    """Build a device scene from host arrays (verts, idx, rgb, light, k_a,
    k_d, background attributes).  Returns the opaque handle (int)."""
    L = load()
    verts = np.ascontiguousarray(scene.verts, dtype=np.float32)
    idx = np.ascontiguousarray(scene.idx, dtype=np.uint32)
    rgb = np.ascontiguousarray(scene.rgb, dtype=np.float32)
    d = rcp_scene_desc()
    d.verts = verts.ctypes.data
    d.n_verts = verts.shape[0]
    d.idx = idx.ctypes.data
    d.n_tris = idx.shape[0]
    d.tri_rgb = rgb.ctypes.data
    d.light_dir[:] = _f3(scene.light)
    d.k_a = float(scene.k_a)
    d.k_d = float(scene.k_d)
    d.background[:] = _f3(scene.background)
    out = ctypes.c_void_p()
    st = L.rcp_build_scene(ctypes.byref(d), ctypes.byref(opts) if opts is not None else None,
                           _stream(stream), ctypes.byref(out))
    _check(st, "rcp_build_scene")
    return out.value


def rcp_destroy_scene(handle: int) -> None:
    load().rcp_destroy_scene(handle)


def rcp_scene_info(handle: int) -> dict:
    s = rcp_scene_stats()
    _check(load().rcp_scene_info(handle, ctypes.byref(s)), "rcp_scene_info")
    return s.as_dict()


def rcp_render(handle: int, cam, W: int, H: int, K: int, disp: rcp_displacement, out_images, out_ids=None,
               stream=None) -> None:
    c = make_camera(cam)
    st = load().rcp_render(handle, ctypes.byref(c), int(W), int(H), int(K), ctypes.byref(disp),
                           _dev_ptr(out_images), _dev_ptr(out_ids), _stream(stream))
    _check(st, "rcp_render")


def rcp_render_noalloc(handle: int, cam, W: int, H: int, K: int, disp: rcp_displacement, out_images, out_ids=None,
                       stream=None) -> None:
    c = make_camera(cam)
    st = load().rcp_render_noalloc(handle, ctypes.byref(c), int(W), int(H), int(K), ctypes.byref(disp),
                                   _dev_ptr(out_images), _dev_ptr(out_ids), _stream(stream))
    _check(st, "rcp_render_noalloc")


def rcp_render_noalloc_scratch_bytes() -> int:
    return int(load().rcp_render_noalloc_scratch_bytes())


def rcp_render_pass(handle: int, cam, W: int, H: int, disp: rcp_displacement, prev_rgb, out_rgb, out_ids=None,
                    stream=None, prev_aux=None, out_aux=None) -> None:
    c = make_camera(cam)
    st = load().rcp_render_pass(handle, ctypes.byref(c), int(W), int(H), ctypes.byref(disp), _dev_ptr(prev_rgb),
                                _dev_ptr(prev_aux), _dev_ptr(out_rgb), _dev_ptr(out_ids), _dev_ptr(out_aux),
                                _stream(stream))
    _check(st, "rcp_render_pass")


def rcp_render_stats(handle: int, cam, W: int, H: int, K: int, disp: rcp_displacement, out_images, out_ids=None,
                     stream=None) -> np.ndarray:
    """Returns uint64 [K][6]: rays traced, inner nodes visited, triangles
    tested, rays continued to the next pass, inner nodes read from LDS, stack
    entries spilled to global memory."""
    c = make_camera(cam)
    counts = np.zeros((K, STAT_COLS), dtype=np.uint64)
    st = load().rcp_render_stats(handle, ctypes.byref(c), int(W), int(H), int(K), ctypes.byref(disp),
                                 _dev_ptr(out_images), _dev_ptr(out_ids), counts.ctypes.data, _stream(stream))
    _check(st, "rcp_render_stats")
    return counts


def rcp_check(handle: int, stream=None) -> None:
    """Synchronise the stream; raise if a ray of an earlier call ran out of
    its traversal step budget."""
    _check(load().rcp_check(handle, _stream(stream)), "rcp_check")


def rcp_debug_set(what: int, value: int) -> None:
    _check(load().rcp_debug_set(int(what), int(value)), "rcp_debug_set")


def rcp_generate_rays(cam, W: int, H: int, disp: rcp_displacement, prev_rgb, out_org, out_dir, stream=None,
                      prev_aux=None) -> None:
    c = make_camera(cam)
    st = load().rcp_generate_rays(ctypes.byref(c), int(W), int(H), ctypes.byref(disp), _dev_ptr(prev_rgb),
                                  _dev_ptr(prev_aux), _dev_ptr(out_org), _dev_ptr(out_dir), _stream(stream))
    _check(st, "rcp_generate_rays")


def rcp_trace_rays(handle: int, org, dirs, n: int, out_t, out_id, out_front=None, stream=None) -> None:
    st = load().rcp_trace_rays(handle, _dev_ptr(org), _dev_ptr(dirs), int(n), _dev_ptr(out_t), _dev_ptr(out_id),
                               _dev_ptr(out_front), _stream(stream))
    _check(st, "rcp_trace_rays")


def rcp_export_bvh(handle: int):
    """Returns (nodes uint32 [n_nodes][node_bytes / 4], tri_ids int32 [n_tris]) on the host."""
    info = rcp_scene_info(handle)
    nodes = np.zeros((info["n_nodes"], info["node_bytes"] // 4), dtype=np.uint32)
    tri_ids = np.zeros(info["n_tris"], dtype=np.int32)
    st = load().rcp_export_bvh(handle, nodes.ctypes.data if nodes.size else None,
                               tri_ids.ctypes.data if tri_ids.size else None)
    _check(st, "rcp_export_bvh")
    return nodes, tri_ids


def rcp_gather_passes(in_rgb, W: int, H: int, n_passes: int, max_smudge: float, edge_mode: int, centred: bool,
                      out_images, stream=None) -> None:
    st = load().rcp_gather_passes(_dev_ptr(in_rgb), int(W), int(H), int(n_passes), float(max_smudge),
                                  int(edge_mode), 1 if centred else 0, _dev_ptr(out_images), _stream(stream))
    _check(st, "rcp_gather_passes")


def rcp_radix_sort_u64(keys, vals, n: int, stream=None) -> None:
    st = load().rcp_radix_sort_u64(_dev_ptr(keys), _dev_ptr(vals), int(n), _stream(stream))
    _check(st, "rcp_radix_sort_u64")


def _view_array(views):
    arr = (rcp_view * len(views))()
    for i, (cam, W, H, K, disp, out, ids) in enumerate(views):
        arr[i].camera = make_camera(cam)
        arr[i].W, arr[i].H, arr[i].K = int(W), int(H), int(K)
        arr[i].disp = disp
        arr[i].out_images = _dev_ptr(out)
        arr[i].out_ids = _dev_ptr(ids)
    return arr


def rcp_render_batch(handle: int, views, stream=None) -> None:
    """views: sequence of (camera, W, H, K, displacement, out_images, out_ids)."""
    st = load().rcp_render_batch(handle, _view_array(views), len(views), _stream(stream))
    _check(st, "rcp_render_batch")


def rcp_autotune_batch(handle: int, views, repeats: int = 3, stream=None):
    """Autotune on a batch (same views as rcp_render_batch); returns
    (tuning dict, median ms of the chosen parameters)."""
    t = rcp_tuning()
    ms = ctypes.c_float()
    st = load().rcp_autotune_batch(handle, _view_array(views), len(views), int(repeats), ctypes.byref(t),
                                   ctypes.byref(ms), _stream(stream))
    _check(st, "rcp_autotune_batch")
    return t.as_dict(), float(ms.value)


def rcp_graph_create(handle: int, cam, W: int, H: int, K: int, disp: rcp_displacement, out_images, out_ids=None,
                     stream=None) -> int:
    c = make_camera(cam)
    out = ctypes.c_void_p()
    st = load().rcp_graph_create(handle, ctypes.byref(c), int(W), int(H), int(K), ctypes.byref(disp),
                                 _dev_ptr(out_images), _dev_ptr(out_ids), _stream(stream), ctypes.byref(out))
    _check(st, "rcp_graph_create")
    return out.value


def rcp_graph_update(graph: int, cam, disp: rcp_displacement) -> None:
    c = make_camera(cam)
    _check(load().rcp_graph_update(graph, ctypes.byref(c), ctypes.byref(disp)), "rcp_graph_update")


def rcp_graph_launch(graph: int, stream=None) -> None:
    _check(load().rcp_graph_launch(graph, _stream(stream)), "rcp_graph_launch")


def rcp_graph_destroy(graph: int) -> None:
    load().rcp_graph_destroy(graph)


def rcp_get_tuning(handle: int) -> dict:
    t = rcp_tuning()
    _check(load().rcp_get_tuning(handle, ctypes.byref(t)), "rcp_get_tuning")
    return t.as_dict()


def rcp_set_tuning(handle: int, refill_min: int | None = None, blocks_per_cu: int | None = None,
                   tile_log2w: int | None = None, engine: int | None = None, exit_lanes: int | None = None,
                   top_levels: int | None = None, stack_entries: int | None = None,
                   block_size: int | None = None, tile_order: int | None = None) -> None:
    """Fields left None keep the scene's current values."""
    t = rcp_tuning(**rcp_get_tuning(handle))
    for k, v in (("refill_min", refill_min), ("blocks_per_cu", blocks_per_cu), ("tile_log2w", tile_log2w),
                 ("engine", engine), ("exit_lanes", exit_lanes), ("top_levels", top_levels),
                 ("stack_entries", stack_entries), ("block_size", block_size), ("tile_order", tile_order)):
        if v is not None:
            setattr(t, k, int(v))
    _check(load().rcp_set_tuning(handle, ctypes.byref(t)), "rcp_set_tuning")


def rcp_autotune(handle: int, cam, W: int, H: int, K: int, disp: rcp_displacement, out_images, out_ids=None,
                 repeats: int = 3, stream=None):
    """Returns (tuning dict, median ms of the chosen parameters)."""
    c = make_camera(cam)
    t = rcp_tuning()
    ms = ctypes.c_float()
    st = load().rcp_autotune(handle, ctypes.byref(c), int(W), int(H), int(K), ctypes.byref(disp),
                             _dev_ptr(out_images), _dev_ptr(out_ids), int(repeats), ctypes.byref(t), ctypes.byref(ms),
                             _stream(stream))
    _check(st, "rcp_autotune")
    return t.as_dict(), float(ms.value)


def autotune_cached(handle: int, scene_key: str, cam, W: int, H: int, K: int, disp: rcp_displacement, out_images,
                    out_ids=None, cache_path: str | None = None, repeats: int = 3, stream=None) -> dict:
    """Tuning for (scene, resolution, K) from a JSON cache, or tuned and
    stored.  The key names the scene (e.g. a digest of its arrays); the
    device name is part of it, since the best parameters depend on the GPU."""
    import json
    import torch
    path = cache_path or os.path.join(os.path.expanduser("~"), ".cache", "rcp_tuning.json")
    key = f"{torch.cuda.get_device_name()}|{scene_key}|{W}x{H}|K{K}|mode{disp.mode}"
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        t = cache[key]["tuning"]
        rcp_set_tuning(handle, **t)
        return t
    t, ms = rcp_autotune(handle, cam, W, H, K, disp, out_images, out_ids, repeats, stream)
    cache[key] = {"tuning": t, "ms": ms}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, path)
    return t


def rcp_server_create(handle: int, pool_bytes: int, max_inflight: int = 2, queue_capacity: int = 1024) -> int:
    out = ctypes.c_void_p()
    _check(load().rcp_server_create(handle, int(pool_bytes), int(max_inflight), int(queue_capacity), ctypes.byref(out)),
           "rcp_server_create")
    return out.value


def rcp_submit(server: int, cam, W: int, H: int, K: int, disp: rcp_displacement, with_ids: bool = False) -> int:
    r = rcp_request()
    r.camera = make_camera(cam)
    r.W, r.H, r.K = int(W), int(H), int(K)
    r.disp = disp
    r.with_ids = 1 if with_ids else 0
    t = ctypes.c_uint64()
    _check(load().rcp_submit(server, ctypes.byref(r), ctypes.byref(t)), "rcp_submit")
    return int(t.value)


def rcp_poll(server: int, ticket: int):
    """Returns (state, (t_submit, t_start, t_done))."""
    state = ctypes.c_int32()
    times = np.zeros(3, np.float64)
    _check(load().rcp_poll(server, int(ticket), ctypes.byref(state), times.ctypes.data), "rcp_poll")
    return int(state.value), tuple(float(x) for x in times)


def rcp_result(server: int, ticket: int):
    """Device addresses (images, ids) of a finished request."""
    a = ctypes.c_void_p()
    b = ctypes.c_void_p()
    _check(load().rcp_result(server, int(ticket), ctypes.byref(a), ctypes.byref(b)), "rcp_result")
    return a.value, b.value


def rcp_result_copy(server: int, ticket: int, images, ids=None, stream=None) -> None:
    _check(load().rcp_result_copy(server, int(ticket), _dev_ptr(images), _dev_ptr(ids), _stream(stream)),
           "rcp_result_copy")


def rcp_release(server: int, ticket: int) -> None:
    _check(load().rcp_release(server, int(ticket)), "rcp_release")


def rcp_server_stats(server: int) -> dict:
    out = np.zeros(4, np.uint64)
    _check(load().rcp_server_stats(server, out.ctypes.data), "rcp_server_stats")
    return {"launches": int(out[0]), "waiting": int(out[1]), "pool_in_use": int(out[2]), "live": int(out[3])}


def rcp_server_destroy(server: int) -> None:
    load().rcp_server_destroy(server)


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------

def build_options(max_leaf: int = 3, c_trav: float = 1.0, c_isect: float = 1.0, builder: int = 0,
                  collapse: int = 0):
    o = rcp_build_options()
    o.max_leaf, o.c_trav, o.c_isect, o.builder = int(max_leaf), float(c_trav), float(c_isect), int(builder)
    o.collapse = int(collapse)
    return o


class Scene:
    """Device scene owned by Python; destroyed with the object."""

    def __init__(self, scene, opts: rcp_build_options | None = None, stream=None):
        self.handle = rcp_build_scene(scene, opts, stream)

    def info(self) -> dict:
        return rcp_scene_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            rcp_destroy_scene(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_engine(self, engine: int) -> None:
        """RCP_ENGINE_CHAIN or RCP_ENGINE_PASSES for rcp_render; the other
        launch parameters stay as they are."""
        rcp_set_tuning(self.handle, engine=engine)

    def render(self, cam, W, H, K, lambda_eye, lambda_dir, with_ids=True, stream=None, mode=RCP_MODE_COLOR,
               z0=0.0):
        """Allocate outputs with torch and render; returns (images, ids)."""
        import torch
        imgs = torch.empty((K, H, W, 3), dtype=torch.float32, device="cuda")
        ids = torch.empty((K, H, W), dtype=torch.int32, device="cuda") if with_ids else None
        rcp_render(self.handle, cam, W, H, K, make_displacement(lambda_eye, lambda_dir, mode, z0), imgs, ids, stream)
        return imgs, ids
