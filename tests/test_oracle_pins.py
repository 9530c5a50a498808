"""Pins for the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself.  Each test checks it against
an independent closed form (plane intersections in float64), an independent
algorithm (Moller-Trumbore in float64 numpy, brute force vs. BVH), or an
invariant the paper states:

* Section 3: the grey seed 0.5 gives no displacement, so the first image is
  the ordinary ray-traced one; average colours do not move rays; R = 1 moves
  right, G = 1 moves up; blue has little effect.
* Section 2: I_n(u,v) depends on I_{n-1}(u,v) only (pointwise), and the
  displacements start from the original positions each pass (not cumulative).
"""
import math

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = []


# ---------------------------------------------------------------------------
# Independent float64 references
# ---------------------------------------------------------------------------

def mt_intersect_all(o, d, tri):
    """Moller-Trumbore in float64 for one ray against all triangles.

    Returns t (inf on miss) and the barycentric margin (min of u, v, 1-u-v).
    """
    v0, v1, v2 = tri[:, 0], tri[:, 1], tri[:, 2]
    e1 = v1 - v0
    e2 = v2 - v0
    p = np.cross(d, e2)
    det = np.einsum("ij,ij->i", e1, p)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        s = o - v0
        u = np.einsum("ij,ij->i", s, p) * inv
        q = np.cross(s, e1)
        v = (q @ d) * inv
        t = np.einsum("ij,ij->i", e2, q) * inv
    margin = np.minimum(np.minimum(u, v), 1.0 - u - v)
    ok = (np.abs(det) > 1e-14) & (margin >= 0) & (t > 0)
    t = np.where(ok, t, np.inf)
    return t, margin


def tri_array(scene):
    return scene.verts.astype(np.float64)[scene.idx.astype(np.int64)]


def pinhole_dir64(cam, W, H, x, y):
    fx = (2 * x + 1) / W - 1.0
    fy = 1.0 - (2 * y + 1) / H
    s = fx * cam.tan_half_fovy * W / H
    t = fy * cam.tan_half_fovy
    q = cam.forward.astype(np.float64) + s * cam.right.astype(np.float64) + t * cam.up.astype(np.float64)
    return q / np.linalg.norm(q), q


AXIS_CAM = scenegen.camera_look_at([0, 0, -3], [0, 0, 0], [0, 1, 0], 60.0)


# ---------------------------------------------------------------------------
# Watertight intersection
# ---------------------------------------------------------------------------

def test_camera_basis_axis_aligned():
    c = AXIS_CAM
    assert np.array_equal(c.right, np.float32([1, 0, 0]))
    assert np.array_equal(c.up, np.float32([0, 1, 0]))
    assert np.array_equal(c.forward, np.float32([0, 0, 1]))


def test_intersect_interior_points_closed_form(oracle_lib):
    rng = np.random.default_rng(123)
    n_ok = 0
    for _ in range(2000):
        tri = rng.uniform(-1, 1, size=(3, 3)).astype(np.float32)
        o = rng.uniform(-3, 3, size=3).astype(np.float32)
        b = rng.dirichlet([1, 1, 1])
        if b.min() < 0.02:
            continue
        target = b @ tri.astype(np.float64)
        d64 = target - o.astype(np.float64)
        d = (d64 / np.linalg.norm(d64)).astype(np.float32)
        n = np.cross(tri[1].astype(np.float64) - tri[0], tri[2].astype(np.float64) - tri[0])
        cosang = abs(np.dot(n, d.astype(np.float64))) / np.linalg.norm(n)
        if cosang < 1e-2:
            continue
        hit, t, front = oracle.intersect(o, d, tri[0], tri[1], tri[2])
        assert hit
        # exact plane intersection of the float32 ray, in float64
        tt = np.dot(n, tri[0].astype(np.float64) - o) / np.dot(n, d.astype(np.float64))
        assert abs(t - tt) <= 1e-5 * max(1.0, abs(tt))
        assert front == (np.dot(n, d.astype(np.float64)) < 0)
        n_ok += 1
    assert n_ok > 1000


def test_intersect_exterior_points_miss(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(1000):
        tri = rng.uniform(-1, 1, size=(3, 3)).astype(np.float32)
        o = rng.uniform(-3, 3, size=3).astype(np.float32)
        b = rng.normal(size=3)
        b = b / b.sum() if abs(b.sum()) > 0.2 else np.array([1.5, -0.25, -0.25])
        if b.min() > -0.02:
            continue
        target = b @ tri.astype(np.float64)
        d64 = target - o
        d = (d64 / np.linalg.norm(d64)).astype(np.float32)
        hit, _, _ = oracle.intersect(o, d, tri[0], tri[1], tri[2])
        assert not hit


def test_intersect_behind_and_parallel_and_degenerate(oracle_lib):
    tri = np.float32([[-1, -1, 2], [1, -1, 2], [0, 1, 2]])
    assert oracle.intersect([0, 0, 0], [0, 0, 1], *tri)[0]
    assert not oracle.intersect([0, 0, 0], [0, 0, -1], *tri)[0]          # behind
    assert not oracle.intersect([0, 0, 2], [0, 0, 1], *tri)[0]           # t == 0 rejected
    assert not oracle.intersect([0, 0, 0], [1, 0, 0], *tri)[0]           # parallel, off-plane
    assert not oracle.intersect([-5, 0, 2], [1, 0, 0], *tri)[0]          # parallel, in-plane
    for deg in ([[0, 0, 2], [1, 1, 2], [2, 2, 2]], [[0, 0, 2], [0, 0, 2], [1, 0, 2]],
                [[0.5, 0.5, 2]] * 3):
        for dx in (0.0, 0.25, 0.5):
            assert not oracle.intersect([dx, dx, 0], [0, 0, 1], *np.float32(deg))[0]


def test_intersect_front_back(oracle_lib):
    tri = np.float32([[-1, -1, 2], [1, -1, 2], [0, 1, 2]])   # normal +z
    hit, t, front = oracle.intersect([0, 0, 0], [0, 0, 1], *tri)
    assert hit and t == 2.0 and front is False
    hit, t, front = oracle.intersect([0, 0, 4], [0, 0, -1], *tri)
    assert hit and t == 2.0 and front is True
    # reversed winding flips the side
    hit, t, front = oracle.intersect([0, 0, 0], [0, 0, 1], tri[0], tri[2], tri[1])
    assert hit and front is True


def test_watertight_shared_edges_and_vertices(oracle_lib):
    """Rays through a shared edge or vertex hit at least one triangle."""
    rng = np.random.default_rng(99)
    for _ in range(300):
        a, b = rng.uniform(-1, 1, size=(2, 3)).astype(np.float32)
        c1, c2 = rng.uniform(-1, 1, size=(2, 3)).astype(np.float32)
        mid = (c1.astype(np.float64) + c2) / 2
        # put c1, c2 on opposite sides of the edge a-b
        ab = b.astype(np.float64) - a
        c2 = (2 * (a + ab * np.dot(mid - a, ab) / np.dot(ab, ab)) - c1).astype(np.float32)
        o = rng.uniform(-4, 4, size=3).astype(np.float32)
        s = rng.uniform(0.05, 0.95)
        p = a.astype(np.float32) + np.float32(s) * (b - a)            # float point on the edge
        d64 = p.astype(np.float64) - o
        d = (d64 / np.linalg.norm(d64)).astype(np.float32)
        h1 = oracle.intersect(o, d, a, b, c1)[0]
        h2 = oracle.intersect(o, d, b, a, c2)[0]
        n = np.cross(ab, c1.astype(np.float64) - a)
        if abs(np.dot(n, d)) / np.linalg.norm(n) < 1e-2:
            continue
        assert h1 or h2
    # a fan sharing the vertex on the axis
    sc = scenegen.adversarial_scene()
    os_ = oracle.OracleScene(sc, use_bvh=False)
    hit, t, tid, _ = os_.closest_hit([0, 0, 0], [0, 0, 1], brute=True)
    assert hit and abs(t - 0.3) < 1e-6


def test_bruteforce_matches_float64_moller_trumbore(oracle_lib):
    """Closest hit (nearest t, then lowest ID) agrees with an independent
    float64 intersector wherever the answer is not decided by rounding."""
    sc = scenegen.soup_scene(3, 200)
    tri = tri_array(sc)
    os_ = oracle.OracleScene(sc, use_bvh=False)
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(3000):
        o = rng.uniform(-2, 2, size=3).astype(np.float32)
        tgt = rng.uniform(-0.5, 0.5, size=3)
        d64 = tgt - o
        d = (d64 / np.linalg.norm(d64)).astype(np.float32)
        t64, margin = mt_intersect_all(o.astype(np.float64), d.astype(np.float64), tri)
        near = np.abs(margin) < 1e-4
        order = np.argsort(t64)
        hit, t, tid, _ = os_.closest_hit(o, d, brute=True)
        if not np.isfinite(t64[order[0]]):
            if near.any():
                continue
            assert not hit
            continue
        best = order[0]
        second = t64[order[1]] if len(order) > 1 else np.inf
        if near.any() or (second - t64[best]) < 1e-4:
            continue
        assert hit and tid == best
        assert abs(t - t64[best]) <= 1e-5 * t64[best]
        checked += 1
    assert checked > 300


@pytest.mark.parametrize("scene_fn", [
    lambda: scenegen.soup_scene(0, 256),
    lambda: scenegen.soup_scene(9, 1500),
    lambda: scenegen.terrain_patch(11, 24, 8),
    lambda: scenegen.adversarial_scene(),
])
def test_bvh_equals_bruteforce(oracle_lib, scene_fn):
    sc = scene_fn()
    ob = oracle.OracleScene(sc, use_bvh=True)
    ofb = oracle.OracleScene(sc, use_bvh=False)
    rng = np.random.default_rng(17)
    lo = sc.verts.min(0)
    hi = sc.verts.max(0)
    ctr = (lo + hi) / 2
    ext = float(np.max(hi - lo))
    for i in range(1500):
        o = (ctr + rng.uniform(-1.5, 1.5, size=3) * ext).astype(np.float32)
        if i % 5 == 0:                       # axis-aligned directions
            d = np.zeros(3, np.float32)
            d[i % 3] = 1.0 if (i // 5) % 2 else -1.0
        else:
            tgt = ctr + rng.uniform(-0.5, 0.5, size=3) * ext
            d = (tgt - o)
            d = (d / np.linalg.norm(d)).astype(np.float32)
        a = ob.closest_hit(o, d, brute=False)
        b = ofb.closest_hit(o, d, brute=True)
        assert a == b, (i, a, b)


# ---------------------------------------------------------------------------
# Rays: pinhole geometry and the colour mapping of Section 3
# ---------------------------------------------------------------------------

def test_pinhole_rays_closed_form(oracle_lib):
    cam = scenegen.camera_look_at([0.1, 0.45, -1.25], [0, 0.05, 0], [0, 1, 0], 60.0)
    for (W, H) in [(64, 64), (1920, 1080), (7, 5)]:
        for (x, y) in [(0, 0), (W - 1, H - 1), (W // 2, H // 3), (W - 1, 0)]:
            o, d = oracle.ray(cam, W, H, x, y, [0.5, 0.5, 0.5], 0.0, 0.01)
            dd, _ = pinhole_dir64(cam, W, H, x, y)
            assert np.array_equal(o, cam.eye)
            assert np.max(np.abs(d - dd)) < 2e-7


def test_seed_gives_undisplaced_ray_for_any_lambda(oracle_lib):
    """I_0 = 0.5 maps to V = 0: the ray is identical for every lambda."""
    cam = scenegen.camera_look_at([0.2, 0.3, -2], [0, 0, 0], [0, 1, 0], 50.0)
    for lam in (0.0, 0.01, 0.3, 0.9):
        o, d = oracle.ray(cam, 33, 17, 5, 11, [0.5, 0.5, 0.5], lam, lam)
        o0, d0 = oracle.ray(cam, 33, 17, 5, 11, [0.5, 0.5, 0.5], 0.0, 0.0)
        assert np.array_equal(o, o0) and np.array_equal(d, d0)


def test_colour_mapping_closed_form(oracle_lib):
    """d ~ q + lambda_dir (2R-1, 2G-1, 2B-1) in (right, up, forward);
    o = eye + lambda_eye (same vector)."""
    cam = scenegen.camera_look_at([0.3, 0.4, -1.7], [0, 0.1, 0], [0, 1, 0], 60.0)
    rng = np.random.default_rng(4)
    M = np.stack([cam.right, cam.up, cam.forward], axis=1).astype(np.float64)   # columns
    for _ in range(200):
        W, H = 97, 61
        x, y = rng.integers(0, W), rng.integers(0, H)
        prev = rng.uniform(0, 1, size=3).astype(np.float32)
        le, ld = rng.uniform(0, 0.3), rng.uniform(0, 0.5)
        o, d = oracle.ray(cam, W, H, int(x), int(y), prev, le, ld)
        m = 2.0 * prev.astype(np.float64) - 1.0
        w = M @ m
        _, q = pinhole_dir64(cam, W, H, x, y)
        dp = q + np.float32(ld) * w
        assert np.max(np.abs(d - dp / np.linalg.norm(dp))) < 1e-6
        assert np.max(np.abs(o - (cam.eye + np.float32(le) * w))) < 1e-6


def test_direction_only_depends_on_difference(oracle_lib):
    """V_e = V_p (lambda_dir = 0): the direction equals the pinhole one bit
    for bit while the eye moves."""
    cam = scenegen.camera_look_at([0, 0.45, -1.25], [0, 0.05, 0], [0, 1, 0], 60.0)
    rng = np.random.default_rng(8)
    for _ in range(100):
        prev = rng.uniform(0, 1, size=3)
        o, d = oracle.ray(cam, 64, 48, 10, 20, prev, 0.05, 0.0)
        o0, d0 = oracle.ray(cam, 64, 48, 10, 20, [0.5, 0.5, 0.5], 0.0, 0.0)
        assert np.array_equal(d, d0)
        assert not np.array_equal(o, o0)


def test_blue_invariant_at_centre_pixel(oracle_lib):
    """With odd W, H the centre ray is the view axis; blue only moves the
    image plane along it, so the direction is unchanged (Section 3: blue has
    little effect)."""
    for b in (0.0, 0.25, 1.0):
        o, d = oracle.ray(AXIS_CAM, 31, 21, 15, 10, [0.5, 0.5, b], 0.0, 0.2)
        assert np.array_equal(d, np.float32([0, 0, 1]))
    # off-centre the footprint scales by 1 / (1 + lambda m_b)
    lam = 0.2
    for b in (0.0, 1.0):
        o, d = oracle.ray(AXIS_CAM, 31, 21, 3, 4, [0.5, 0.5, b], 0.0, lam)
        _, q = pinhole_dir64(AXIS_CAM, 31, 21, 3, 4)
        mb = 2 * b - 1
        assert abs(d[0] / d[2] - q[0] / (1 + lam * mb)) < 1e-6
        assert abs(d[1] / d[2] - q[1] / (1 + lam * mb)) < 1e-6


def _stripes_scene(axis: int, width: float = 0.02, half: float = 4.0):
    """Plane z = 0 cut into thin stripes along x (axis 0) or y (axis 1)."""
    n = int(round(2 * half / width))
    vs, ts = [], []
    for i in range(n):
        a = -half + i * width
        b = a + width
        if axis == 0:
            quad = [[a, -half, 0], [b, -half, 0], [b, half, 0], [a, half, 0]]
        else:
            quad = [[-half, a, 0], [half, a, 0], [half, b, 0], [-half, b, 0]]
        base = len(vs)
        vs += quad
        ts += [[base, base + 2, base + 1], [base, base + 3, base + 2]]
    rgb = np.tile(np.float32([0.7, 0.5, 0.5]), (len(ts), 1))
    return scenegen.Scene(verts=np.array(vs), idx=np.array(ts), rgb=rgb, name="stripes"), n, half, width


@pytest.mark.parametrize("axis,prev", [(0, (1.0, 0.5, 0.5)), (0, (0.0, 0.5, 0.5)),
                                       (1, (0.5, 1.0, 0.5)), (1, (0.5, 0.0, 0.5))])
def test_red_right_green_up(oracle_lib, axis, prev):
    """Section 3: R = 1 moves the sample right, R = 0 left; G = 1 up, G = 0
    down.  The stripe hit by each displaced ray matches the float64 closed
    form of the displaced ray's intersection with the plane z = 0."""
    sc, n, half, width = _stripes_scene(axis)
    os_ = oracle.OracleScene(sc, use_bvh=True)
    W, H, lam = 41, 29, 0.05
    img_prev = np.tile(np.float32(prev), (H, W, 1))
    out, ids = os_.render_pass(AXIS_CAM, W, H, 0.0, lam, prev=img_prev)
    out0, ids0 = os_.render_pass(AXIS_CAM, W, H, 0.0, lam, prev=None)
    m = 2 * np.float64(prev) - 1
    shifted = 0
    for y in range(H):
        for x in range(W):
            _, q = pinhole_dir64(AXIS_CAM, W, H, x, y)
            dp = q + lam * m          # the camera frame is the world frame here
            hit = AXIS_CAM.eye.astype(np.float64) + (3.0 / dp[2]) * dp
            coord = hit[axis]
            k = (coord + half) / width
            if abs(k - round(k)) < 1e-3:
                continue
            assert ids[y, x] // 2 == int(math.floor(k)), (x, y)
            # compared with the undisplaced pass, the stripe index moved by
            # lambda * 3 / width = 7.5 stripes in the direction of m
            shifted += 1
            assert np.sign(ids[y, x] // 2 - ids0[y, x] // 2) == np.sign(m[axis])
    assert shifted > W * H // 2


# ---------------------------------------------------------------------------
# Pinhole render of an analytic scene, shading
# ---------------------------------------------------------------------------

def test_quad_pinhole_render_closed_form(oracle_lib):
    sc = scenegen.quad_scene(z0=0.0, half=0.8, rgb=(0.8, 0.6, 0.4))
    os_ = oracle.OracleScene(sc, use_bvh=True)
    W, H = 45, 37
    img, ids = os_.render_pass(AXIS_CAM, W, H, 0.0, 0.02, prev=None)
    L = np.array([0.3, 0.8, -0.5]) / math.sqrt(0.98)
    shade = max(0.0, float(np.dot([0, 0, -1], L)))           # quad normal faces the camera
    want = np.array([0.8, 0.6, 0.4]) * shade
    n_hit = 0
    for y in range(H):
        for x in range(W):
            dd, _ = pinhole_dir64(AXIS_CAM, W, H, x, y)
            t = 3.0 / dd[2]
            px, py = t * dd[0], t * dd[1]
            inside = max(abs(px), abs(py)) < 0.8 - 1e-5
            outside = max(abs(px), abs(py)) > 0.8 + 1e-5
            if inside:
                assert ids[y, x] in (0, 1)
                assert np.max(np.abs(img[y, x] - want)) < 2e-7
                n_hit += 1
            elif outside:
                assert ids[y, x] == -1
                assert np.array_equal(img[y, x], sc.background)
    assert n_hit > 0


def test_lambert_shade_hand_values(oracle_lib):
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=np.float32)   # normal +z
    sc = scenegen.Scene(verts=tri, idx=[[0, 1, 2]], rgb=[[0.5, 1.0, 0.25]],
                        light=np.float32([0, 0.6, 0.8]), k_a=0.1, k_d=0.9)
    os_ = oracle.OracleScene(sc, use_bvh=False)
    # front (normal +z toward the viewer): dot = 0.8
    f = os_.shade(0, True)
    s = np.float32(0.1) + np.float32(0.9) * np.float32(0.8)
    assert np.allclose(f, np.float32([0.5, 1.0, 0.25]) * s, atol=1e-7)
    # back: normal -z, dot = -0.8 -> ambient only
    b = os_.shade(0, False)
    assert np.allclose(b, np.float32([0.5, 1.0, 0.25]) * np.float32(0.1), atol=1e-7)
    # clamp to [0, 1]
    sc2 = scenegen.Scene(verts=tri, idx=[[0, 1, 2]], rgb=[[1.0, 0.9, 0.2]],
                         light=np.float32([0, 0, 1]), k_a=0.5, k_d=1.0)
    c = oracle.OracleScene(sc2, use_bvh=False).shade(0, True)
    assert c[0] == 1.0 and c[1] == 1.0 and abs(c[2] - 0.3) < 1e-7


# ---------------------------------------------------------------------------
# Recursion structure (Section 2)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def soup():
    w = scenegen.workload("soup256")
    return w, oracle.OracleScene(w.scene, use_bvh=True)


@pytest.fixture(scope="module")
def patch():
    sc = scenegen.terrain_patch(11, 24, 8)
    cam = scenegen.camera_look_at([0, 0.5, -1.4], [0, 0.05, 0], [0, 1, 0], 60.0)
    return sc, cam, oracle.OracleScene(sc, use_bvh=True)


def test_average_colour_does_not_move_rays(oracle_lib, patch):
    sc, cam, os_ = patch
    W, H = 40, 30
    a, ia = os_.render_pass(cam, W, H, 0.0, 0.05, prev=None)
    b, ib = os_.render_pass(cam, W, H, 0.0, 0.05, prev=np.full((H, W, 3), 0.5, np.float32))
    assert np.array_equal(a, b) and np.array_equal(ia, ib)


def test_lambda_zero_all_passes_equal(oracle_lib, patch):
    sc, cam, os_ = patch
    img, ids = os_.render(cam, 32, 24, 4, 0.0, 0.0)
    for k in range(1, 4):
        assert np.array_equal(img[k], img[0]) and np.array_equal(ids[k], ids[0])


def test_first_image_independent_of_lambda(oracle_lib, patch):
    sc, cam, os_ = patch
    a, ia = os_.render(cam, 32, 24, 2, 0.0, 0.0)
    b, ib = os_.render(cam, 32, 24, 2, 0.04, 0.04)
    assert np.array_equal(a[0], b[0]) and np.array_equal(ia[0], ib[0])
    assert not np.array_equal(a[1], b[1])


def test_pointwise_dependence(oracle_lib, patch):
    sc, cam, os_ = patch
    W, H = 36, 28
    img, _ = os_.render(cam, W, H, 2, 0.0, 0.05)
    prev = img[0].copy()
    base, _ = os_.render_pass(cam, W, H, 0.0, 0.05, prev=prev)
    rng = np.random.default_rng(1)
    for _ in range(10):
        y, x = rng.integers(0, H), rng.integers(0, W)
        p2 = prev.copy()
        p2[y, x] = rng.uniform(0, 1, size=3)
        out, _ = os_.render_pass(cam, W, H, 0.0, 0.05, prev=p2)
        diff = np.any(out != base, axis=-1)
        diff[y, x] = False
        assert not diff.any()


def test_chain_equals_repeated_single_passes(oracle_lib, patch):
    """Each pass displaces the ORIGINAL camera using only the previous image."""
    sc, cam, os_ = patch
    W, H, K = 30, 22, 5
    img, ids = os_.render(cam, W, H, K, 0.01, 0.05)
    prev = None
    for k in range(K):
        out, oid = os_.render_pass(cam, W, H, 0.01, 0.05, prev=prev)
        assert np.array_equal(out, img[k]) and np.array_equal(oid, ids[k])
        prev = out


def test_prefix_stability(oracle_lib, soup):
    w, os_ = soup
    a, ia = os_.render(w.camera, 64, 64, 6, 0.0, 0.02)
    b, ib = os_.render(w.camera, 64, 64, 3, 0.0, 0.02)
    assert np.array_equal(a[:3], b) and np.array_equal(ia[:3], ib)


def test_pixel_chains_equal_full_render(oracle_lib, patch):
    sc, cam, os_ = patch
    W, H, K = 50, 35, 4
    img, ids = os_.render(cam, W, H, K, 0.0, 0.05)
    rng = np.random.default_rng(3)
    pix = rng.choice(W * H, size=200, replace=False).astype(np.int32)
    out, oid = os_.render_pixels(cam, W, H, K, 0.0, 0.05, pix)
    ys, xs = pix // W, pix % W
    assert np.array_equal(out, img[:, ys, xs].transpose(1, 0, 2))
    assert np.array_equal(oid, ids[:, ys, xs].T)


def test_thread_count_does_not_change_result(oracle_lib, soup):
    w, os_ = soup
    a, ia = os_.render(w.camera, 64, 64, 3, 0.0, 0.02, nthreads=1)
    b, ib = os_.render(w.camera, 64, 64, 3, 0.0, 0.02, nthreads=5)
    assert np.array_equal(a, b) and np.array_equal(ia, ib)


def test_displaced_passes_differ_and_stay_ldr(oracle_lib, patch):
    """Fig. 2 shows every displaced pass smudged relative to the first; the
    channels stay in the low dynamic range [0, 1] (Section 3)."""
    sc, cam, os_ = patch
    img, _ = os_.render(cam, 64, 48, 6, 0.0, 0.03)
    d = [float(np.mean(np.abs(img[k] - img[0]))) for k in range(6)]
    assert d[0] == 0.0 and min(d[1:]) > 0.0
    assert img.min() >= 0.0 and img.max() <= 1.0


@pytest.mark.parametrize("W,H,eye", [(67, 45, [0, 0.5, -1.4]), (33, 33, [0, 0.3, -2.0]), (64, 48, [0.25, 0.6, -1.2])])
def test_bvh_equals_bruteforce_on_grid_plane_rays(oracle_lib, W, H, eye):
    """Camera rays whose direction has an exactly zero component and that lie
    in a grid plane of the terrain (odd W: the centre column is the plane
    x = 0) hit two triangles at the same t; the lower index must win through
    the BVH exactly as in the brute-force scan."""
    sc = scenegen.terrain_patch(11, 24, 8)
    cam = scenegen.camera_look_at(eye, [eye[0], 0.05, 0], [0, 1, 0], 60.0)
    a, ia = oracle.OracleScene(sc, use_bvh=True).render(cam, W, H, 3, 0.0, 0.05)
    b, ib = oracle.OracleScene(sc, use_bvh=False).render(cam, W, H, 3, 0.0, 0.05)
    assert np.array_equal(a, b) and np.array_equal(ia, ib)
