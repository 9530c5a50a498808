"""CPU oracle for recursive camera painting -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct implementation of the K-pass render written
from the paper (Section 2: per-(u,v) recursion and ray definition; Section 3:
colour-driven displacement).  It is compiled from ``rcp_oracle.c`` with gcc
(``-O2 -ffp-contract=off``) and driven through ctypes.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the HIP library; the only common input
is the seeded scene data produced by ``scenegen``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rcp_oracle.c")
_LIB = os.path.join(_HERE, "librcp_oracle.so")
# A test that plants a mistake in a copy of the oracle points this at the
# copy's library; nothing else sets it.
_LIB_OVERRIDE = os.environ.get("RCP_ORACLE_LIB")

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-pthread", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile the oracle shared library in place; returns its path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("n_verts", ctypes.c_uint32),
                ("idx", ctypes.c_void_p), ("n_tris", ctypes.c_uint32),
                ("rgb", ctypes.c_void_p), ("light", ctypes.c_float * 3),
                ("k_a", ctypes.c_float), ("k_d", ctypes.c_float),
                ("background", ctypes.c_float * 3)]


class _Cam(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("right", ctypes.c_float * 3),
                ("up", ctypes.c_float * 3), ("forward", ctypes.c_float * 3),
                ("tan_half_fovy", ctypes.c_float)]


MODE_COLOR, MODE_DEPTH, MODE_NORMAL = 0, 1, 2
EDGE_CLAMP, EDGE_WRAP, EDGE_MIRROR = 0, 1, 2

_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            path = _LIB_OVERRIDE
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        f32 = ctypes.c_float
        i32 = ctypes.c_int
        L.orc_scene_create.restype = P
        L.orc_scene_create.argtypes = [ctypes.POINTER(_Desc), i32]
        L.orc_scene_destroy.argtypes = [P]
        L.orc_scene_stats.argtypes = [P, P]
        L.orc_ray.argtypes = [ctypes.POINTER(_Cam), i32, i32, i32, i32, P, P, i32, f32, f32, f32, P, P]
        L.orc_intersect.restype = i32
        L.orc_intersect.argtypes = [P, P, P, P, P, P, P]
        L.orc_closest_hit.restype = i32
        L.orc_closest_hit.argtypes = [P, P, P, i32, P, P, P]
        L.orc_closest_hits.restype = i32
        L.orc_closest_hits.argtypes = [P, P, P, i32, i32, P, P, P, i32]
        L.orc_shade.argtypes = [P, ctypes.c_int32, i32, P]
        L.orc_normal.argtypes = [P, ctypes.c_int32, P]
        L.orc_render_pass.restype = i32
        L.orc_render_pass.argtypes = [P, ctypes.POINTER(_Cam), i32, i32, i32, f32, f32, f32, P, P, P, P, P, i32]
        L.orc_render.restype = i32
        L.orc_render.argtypes = [P, ctypes.POINTER(_Cam), i32, i32, i32, i32, f32, f32, f32, P, P, i32]
        L.orc_render_pixels.restype = i32
        L.orc_render_pixels.argtypes = [P, ctypes.POINTER(_Cam), i32, i32, i32, i32, f32, f32, f32, P, i32,
                                        P, P, i32]
        L.orc_default_threads.restype = i32
        L.orc_gather.restype = i32
        L.orc_gather.argtypes = [P, i32, i32, i32, f32, i32, i32, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f3(a):
    return np.ascontiguousarray(a, dtype=np.float32).reshape(3)


def camera_struct(cam) -> _Cam:
    c = _Cam()
    for k in ("eye", "right", "up", "forward"):
        getattr(c, k)[:] = [float(x) for x in _f3(getattr(cam, k))]
    c.tan_half_fovy = float(np.float32(cam.tan_half_fovy))
    return c


class OracleScene:
    """Scene copied into the oracle, with (use_bvh=True) its own SAH BVH."""

    def __init__(self, scene, use_bvh: bool = True):
        L = lib()
        self._keep = (np.ascontiguousarray(scene.verts, np.float32),
                      np.ascontiguousarray(scene.idx, np.uint32),
                      np.ascontiguousarray(scene.rgb, np.float32))
        d = _Desc()
        d.verts = _ptr(self._keep[0])
        d.n_verts = self._keep[0].shape[0]
        d.idx = _ptr(self._keep[1])
        d.n_tris = self._keep[1].shape[0]
        d.rgb = _ptr(self._keep[2])
        d.light[:] = [float(x) for x in _f3(scene.light)]
        d.k_a = float(scene.k_a)
        d.k_d = float(scene.k_d)
        d.background[:] = [float(x) for x in _f3(scene.background)]
        self.h = L.orc_scene_create(ctypes.byref(d), 1 if use_bvh else 0)
        if not self.h:
            raise ValueError("oracle rejected the scene")
        self.scene = scene

    def close(self):
        if getattr(self, "h", None):
            lib().orc_scene_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        out = np.zeros(3, np.int32)
        lib().orc_scene_stats(self.h, _ptr(out))
        return {"nodes": int(out[0]), "leaves": int(out[1]), "max_depth": int(out[2])}

    def closest_hit(self, o, d, brute: bool = False):
        o = _f3(o); d = _f3(d)
        t = np.zeros(1, np.float32); i = np.zeros(1, np.int32); f = np.zeros(1, np.int32)
        hit = lib().orc_closest_hit(self.h, _ptr(o), _ptr(d), 1 if brute else 0, _ptr(t), _ptr(i), _ptr(f))
        return (True, float(t[0]), int(i[0]), bool(f[0])) if hit else (False, None, -1, None)

    def closest_hits(self, o, d, brute: bool = False, nthreads: int = 0):
        """Closest hits of rays o[n][3], d[n][3]: (t [n] with +inf on a miss,
        id [n] with -1 on a miss, front [n] bool)."""
        o = np.ascontiguousarray(o, np.float32).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float32).reshape(-1, 3)
        n = o.shape[0]
        t = np.zeros(n, np.float32); i = np.zeros(n, np.int32); f = np.zeros(n, np.int32)
        rc = lib().orc_closest_hits(self.h, _ptr(o), _ptr(d), n, 1 if brute else 0, _ptr(t), _ptr(i), _ptr(f),
                                    int(nthreads))
        if rc:
            raise ValueError("orc_closest_hits failed")
        return t, i, f.astype(bool)

    def shade(self, tri_id: int, front: bool):
        out = np.zeros(3, np.float32)
        lib().orc_shade(self.h, int(tri_id), 1 if front else 0, _ptr(out))
        return out

    def normal(self, tri_id: int):
        out = np.zeros(3, np.float32)
        lib().orc_normal(self.h, int(tri_id), _ptr(out))
        return out

    def render_pass(self, cam, W, H, lambda_eye, lambda_dir, prev=None, prev_aux=None, mode=MODE_COLOR,
                    z0=0.0, nthreads=0, with_aux=False):
        """One pass; returns (image, ids) or (image, ids, aux) with with_aux."""
        out = np.zeros((H, W, 3), np.float32)
        ids = np.zeros((H, W), np.int32)
        aux = np.zeros((H, W, 4), np.float32)
        p = None if prev is None else np.ascontiguousarray(prev, np.float32).reshape(H, W, 3)
        pa = None if prev_aux is None else np.ascontiguousarray(prev_aux, np.float32).reshape(H, W, 4)
        c = camera_struct(cam)
        rc = lib().orc_render_pass(self.h, ctypes.byref(c), W, H, int(mode), float(z0), float(lambda_eye),
                                   float(lambda_dir), _ptr(p), _ptr(pa), _ptr(out), _ptr(ids), _ptr(aux),
                                   int(nthreads))
        if rc:
            raise ValueError("orc_render_pass failed")
        return (out, ids, aux) if with_aux else (out, ids)

    def render(self, cam, W, H, K, lambda_eye, lambda_dir, nthreads=0, mode=MODE_COLOR, z0=0.0):
        out = np.zeros((K, H, W, 3), np.float32)
        ids = np.zeros((K, H, W), np.int32)
        c = camera_struct(cam)
        rc = lib().orc_render(self.h, ctypes.byref(c), W, H, K, int(mode), float(z0), float(lambda_eye),
                              float(lambda_dir), _ptr(out), _ptr(ids), int(nthreads))
        if rc:
            raise ValueError("orc_render failed")
        return out, ids

    def render_pixels(self, cam, W, H, K, lambda_eye, lambda_dir, pix, nthreads=0, mode=MODE_COLOR, z0=0.0):
        pix = np.ascontiguousarray(pix, np.int32).reshape(-1)
        out = np.zeros((pix.shape[0], K, 3), np.float32)
        ids = np.zeros((pix.shape[0], K), np.int32)
        c = camera_struct(cam)
        rc = lib().orc_render_pixels(self.h, ctypes.byref(c), W, H, K, int(mode), float(z0), float(lambda_eye),
                                     float(lambda_dir), _ptr(pix), pix.shape[0], _ptr(out), _ptr(ids),
                                     int(nthreads))
        if rc:
            raise ValueError("orc_render_pixels failed")
        return out, ids


def ray(cam, W, H, x, y, prev, lambda_eye, lambda_dir, prev_aux=None, mode=MODE_COLOR, z0=0.0):
    o = np.zeros(3, np.float32); d = np.zeros(3, np.float32)
    p = _f3(prev)
    pa = None if prev_aux is None else np.ascontiguousarray(prev_aux, np.float32).reshape(4)
    c = camera_struct(cam)
    lib().orc_ray(ctypes.byref(c), W, H, x, y, _ptr(p), _ptr(pa), int(mode), float(z0), float(lambda_eye),
                  float(lambda_dir), _ptr(o), _ptr(d))
    return o, d


def intersect(o, d, v0, v1, v2):
    arr = [_f3(x) for x in (o, d, v0, v1, v2)]
    t = np.zeros(1, np.float32); f = np.zeros(1, np.int32)
    hit = lib().orc_intersect(*[_ptr(a) for a in arr], _ptr(t), _ptr(f))
    return (True, float(t[0]), bool(f[0])) if hit else (False, None, None)


def default_threads() -> int:
    return int(lib().orc_default_threads())


def gather(img, n, max_smudge, edge=EDGE_MIRROR, centred=True):
    """n screen-space passes starting from img [H][W][3]; returns [n][H][W][3]."""
    img = np.ascontiguousarray(img, np.float32)
    H, W = img.shape[:2]
    out = np.zeros((n, H, W, 3), np.float32)
    rc = lib().orc_gather(_ptr(img), W, H, int(n), float(max_smudge), int(edge), 1 if centred else 0, _ptr(out))
    if rc:
        raise ValueError("orc_gather failed")
    return out
