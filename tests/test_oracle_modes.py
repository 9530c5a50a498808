"""Pins for the oracle's depth (Section 4) and normal (Section 5) mappings.

Depth: V_p = lambda |z - z0| (2I - 1), z the view depth of the previous hit.
Normal: V_p = lambda (C x N), C the pixel's view direction, N the world
normal of the previous hit.  Each check is against a float64 closed form or
an invariant of those definitions, never the oracle itself.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen
from test_oracle_pins import AXIS_CAM, _stripes_scene, pinhole_dir64

DEPTH, NORMAL = oracle.MODE_DEPTH, oracle.MODE_NORMAL


def test_seed_gives_pinhole_rays_in_every_mode(oracle_lib):
    cam = scenegen.camera_look_at([0.2, 0.3, -2], [0, 0, 0], [0, 1, 0], 50.0)
    for mode in (DEPTH, NORMAL):
        o, d = oracle.ray(cam, 33, 17, 5, 11, [0.9, 0.1, 0.7], 0.05, 0.2, prev_aux=None, mode=mode, z0=1.0)
        o0, d0 = oracle.ray(cam, 33, 17, 5, 11, [0.5, 0.5, 0.5], 0.0, 0.0)
        if mode == NORMAL:
            assert np.array_equal(o, o0) and np.array_equal(d, d0)
        else:
            # no depth yet (the seed has no hit): no displacement either
            assert np.array_equal(o, o0) and np.array_equal(d, d0)


def test_depth_in_focus_and_miss_are_not_displaced(oracle_lib):
    cam = scenegen.camera_look_at([0.3, 0.4, -1.7], [0, 0.1, 0], [0, 1, 0], 60.0)
    rng = np.random.default_rng(2)
    for _ in range(50):
        prev = rng.uniform(0, 1, 3)
        z0 = float(rng.uniform(0.5, 3))
        x, y = int(rng.integers(0, 40)), int(rng.integers(0, 30))
        o0, d0 = oracle.ray(cam, 40, 30, x, y, [0.5, 0.5, 0.5], 0.0, 0.0)
        o, d = oracle.ray(cam, 40, 30, x, y, prev, 0.1, 0.3, prev_aux=[z0, 0, 1, 0], mode=DEPTH, z0=z0)
        assert np.array_equal(d, d0) and np.array_equal(o, o0)
        o, d = oracle.ray(cam, 40, 30, x, y, prev, 0.1, 0.3, prev_aux=[np.inf, 0, 0, 0], mode=DEPTH, z0=z0)
        assert np.array_equal(d, d0) and np.array_equal(o, o0)


def test_depth_mapping_closed_form(oracle_lib):
    cam = scenegen.camera_look_at([0.3, 0.4, -1.7], [0, 0.1, 0], [0, 1, 0], 60.0)
    M = np.stack([cam.right, cam.up, cam.forward], axis=1).astype(np.float64)
    rng = np.random.default_rng(4)
    for _ in range(200):
        W, H = 57, 41
        x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        prev = rng.uniform(0, 1, 3).astype(np.float32)
        z, z0 = float(rng.uniform(0.5, 4)), float(rng.uniform(0.5, 4))
        le, ld = float(rng.uniform(0, 0.1)), float(rng.uniform(0, 0.3))
        o, d = oracle.ray(cam, W, H, x, y, prev, le, ld, prev_aux=[z, 0, 0, 0], mode=DEPTH, z0=z0)
        w = abs(np.float32(z) - np.float32(z0)) * (M @ (2.0 * prev.astype(np.float64) - 1.0))
        _, q = pinhole_dir64(cam, W, H, x, y)
        dp = q + np.float32(ld) * w
        assert np.max(np.abs(d - dp / np.linalg.norm(dp))) < 2e-6
        assert np.max(np.abs(o - (cam.eye + np.float32(le) * w))) < 2e-6


def test_normal_mapping_closed_form(oracle_lib):
    cam = scenegen.camera_look_at([0.3, 0.4, -1.7], [0, 0.1, 0], [0, 1, 0], 60.0)
    rng = np.random.default_rng(5)
    for _ in range(200):
        W, H = 57, 41
        x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        n = rng.normal(size=3)
        n = (n / np.linalg.norm(n)).astype(np.float32)
        le, ld = float(rng.uniform(0, 0.1)), float(rng.uniform(0, 0.3))
        o, d = oracle.ray(cam, W, H, x, y, [0.5, 0.5, 0.5], le, ld, prev_aux=[1.0, *n], mode=NORMAL)
        dd, q = pinhole_dir64(cam, W, H, x, y)
        w = np.cross(dd, n.astype(np.float64))
        dp = q + np.float32(ld) * w
        assert np.max(np.abs(d - dp / np.linalg.norm(dp))) < 2e-6
        assert np.max(np.abs(o - (cam.eye + np.float32(le) * w))) < 2e-6


def test_normal_parallel_to_view_does_not_move_the_ray(oracle_lib):
    for nz in (1.0, -1.0):
        o, d = oracle.ray(AXIS_CAM, 31, 21, 15, 10, [0.5, 0.5, 0.5], 0.0, 0.4, prev_aux=[2.0, 0, 0, nz], mode=NORMAL)
        assert np.array_equal(d, np.float32([0, 0, 1]))


@pytest.mark.parametrize("mode,aux,axis,sign,scale", [
    (DEPTH, [5.0, 0, 0, 0], 0, +1, 2.0),      # colour R = 1 at |5 - 3| = 2: twice the colour shift, right
    (DEPTH, [3.5, 0, 0, 0], 0, +1, 0.5),
    (NORMAL, [3.0, 0, 1, 0], 0, -1, 1.0),     # C ~ +z, N = +y: C x N ~ -x (left)
    (NORMAL, [3.0, 1, 0, 0], 1, +1, 1.0),     # C ~ +z, N = +x: C x N ~ +y (up)
])
def test_modes_move_samples_as_the_closed_form_says(oracle_lib, mode, aux, axis, sign, scale):
    sc, n, half, width = _stripes_scene(axis)
    os_ = oracle.OracleScene(sc, use_bvh=True)
    W, H, lam = 41, 29, 0.05
    prev = np.tile(np.float32([1.0, 0.5, 0.5]), (H, W, 1))
    prev_aux = np.tile(np.float32(aux), (H, W, 1))
    out, ids = os_.render_pass(AXIS_CAM, W, H, 0.0, lam, prev=prev, prev_aux=prev_aux, mode=mode, z0=3.0)
    checked = 0
    for y in range(H):
        for x in range(W):
            dd, q = pinhole_dir64(AXIS_CAM, W, H, x, y)
            if mode == DEPTH:
                w = abs(aux[0] - 3.0) * np.array([1.0, 0.0, 0.0])
            else:
                w = np.cross(dd, np.array(aux[1:], dtype=np.float64))
            dp = q + lam * w
            hit = AXIS_CAM.eye.astype(np.float64) + (3.0 / dp[2]) * dp
            k = (hit[axis] + half) / width
            if abs(k - round(k)) < 1e-3:
                continue
            assert ids[y, x] // 2 == int(math.floor(k)), (x, y)
            checked += 1
            # the displacement at the plane: lambda * scale * 3 (distance) units
            k0 = (AXIS_CAM.eye[axis] + 3.0 * q[axis] / q[2] + half) / width
            assert np.sign(k - k0) == sign
            if mode == DEPTH:
                assert abs((k - k0) * width - sign * lam * scale * 3.0) < 1e-9
    assert checked > W * H // 2


def test_aux_is_view_depth_and_unit_normal(oracle_lib):
    sc = scenegen.quad_scene(z0=0.0, half=0.8)
    os_ = oracle.OracleScene(sc, use_bvh=False)
    W, H = 31, 23
    _, ids, aux = os_.render_pass(AXIS_CAM, W, H, 0.0, 0.0, with_aux=True)
    hit = ids >= 0
    assert hit.any() and (~hit).any()
    assert np.all(np.abs(aux[hit][:, 0] - 3.0) < 1e-6)          # plane z = 0 seen from z = -3
    assert np.array_equal(aux[hit][:, 1:], np.tile(np.float32([0, 0, -1]), (int(hit.sum()), 1)))
    assert np.all(np.isinf(aux[~hit][:, 0])) and np.all(aux[~hit][:, 1:] == 0)
    # a tilted triangle: normal against the float64 cross product, depth against the plane
    tri = np.array([[-1, -1, 1.0], [1, -1, 2.0], [0, 1, 1.5]], dtype=np.float32)
    sc2 = scenegen.Scene(verts=tri, idx=[[0, 1, 2]], rgb=[[0.5, 0.5, 0.5]])
    o2 = oracle.OracleScene(sc2, use_bvh=False)
    n64 = np.cross(tri[1].astype(np.float64) - tri[0], tri[2].astype(np.float64) - tri[0])
    assert np.allclose(o2.normal(0), n64 / np.linalg.norm(n64), atol=1e-7)
    _, ids2, aux2 = o2.render_pass(AXIS_CAM, 21, 21, 0.0, 0.0, with_aux=True)
    for y, x in zip(*np.nonzero(ids2 >= 0)):
        dd, _ = pinhole_dir64(AXIS_CAM, 21, 21, x, y)
        t = np.dot(n64, tri[0].astype(np.float64) - AXIS_CAM.eye) / np.dot(n64, dd)
        assert abs(aux2[y, x, 0] - t * dd[2]) < 1e-5


@pytest.fixture(scope="module")
def patch():
    sc = scenegen.terrain_patch(11, 24, 8)
    cam = scenegen.camera_look_at([0, 0.5, -1.4], [0, 0.05, 0], [0, 1, 0], 60.0)
    return sc, cam, oracle.OracleScene(sc, use_bvh=True)


@pytest.mark.parametrize("mode", [DEPTH, NORMAL])
def test_mode_chain_equals_repeated_passes(oracle_lib, patch, mode):
    sc, cam, os_ = patch
    W, H, K = 30, 22, 5
    img, ids = os_.render(cam, W, H, K, 0.01, 0.05, mode=mode, z0=1.2)
    prev, prev_aux = None, None
    for k in range(K):
        out, oid, aux = os_.render_pass(cam, W, H, 0.01, 0.05, prev=prev, prev_aux=prev_aux, mode=mode, z0=1.2,
                                        with_aux=True)
        assert np.array_equal(out, img[k]) and np.array_equal(oid, ids[k])
        prev, prev_aux = out, aux
    assert not np.array_equal(img[0], img[-1])


@pytest.mark.parametrize("mode", [DEPTH, NORMAL])
def test_mode_pointwise_and_pixel_chains(oracle_lib, patch, mode):
    sc, cam, os_ = patch
    W, H, K = 36, 28, 4
    img, ids = os_.render(cam, W, H, K, 0.0, 0.05, mode=mode, z0=1.2)
    rng = np.random.default_rng(3)
    pix = rng.choice(W * H, size=150, replace=False).astype(np.int32)
    out, oid = os_.render_pixels(cam, W, H, K, 0.0, 0.05, pix, mode=mode, z0=1.2)
    ys, xs = pix // W, pix % W
    assert np.array_equal(out, img[:, ys, xs].transpose(1, 0, 2))
    assert np.array_equal(oid, ids[:, ys, xs].T)
    _, _, aux0 = os_.render_pass(cam, W, H, 0.0, 0.05, mode=mode, z0=1.2, with_aux=True)
    base, _ = os_.render_pass(cam, W, H, 0.0, 0.05, prev=img[0], prev_aux=aux0, mode=mode, z0=1.2)
    for _ in range(6):
        y, x = int(rng.integers(0, H)), int(rng.integers(0, W))
        a2 = aux0.copy()
        a2[y, x] = [0.3, 0.6, 0.0, 0.8]
        p2 = img[0].copy()
        p2[y, x] = [1.0, 0.0, 1.0]
        out2, _ = os_.render_pass(cam, W, H, 0.0, 0.05, prev=p2, prev_aux=a2, mode=mode, z0=1.2)
        diff = np.any(out2 != base, axis=-1)
        diff[y, x] = False
        assert not diff.any()


@pytest.mark.parametrize("mode", [DEPTH, NORMAL])
def test_mode_lambda_zero_all_passes_equal(oracle_lib, patch, mode):
    sc, cam, os_ = patch
    img, ids = os_.render(cam, 32, 24, 3, 0.0, 0.0, mode=mode, z0=1.0)
    assert np.array_equal(img[1], img[0]) and np.array_equal(img[2], img[0])
