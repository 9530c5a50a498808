"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every case runs both sides on the same seeded inputs.  The bar (written in
``_parity.py``): pass-1 hit IDs bit-exact; after the K passes mean |dRGB| <=
1e-3 and <= 0.1% of pixels with a channel off by more than 1/255.  Ray
generation and the closest-hit query are compared bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from _parity import assert_parity
from paper_2312_12392_amd import rcp

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    rcp.load()


ENGINES = [rcp.RCP_ENGINE_CHAIN, rcp.RCP_ENGINE_PASSES]
ENGINE_IDS = ["chain", "passes"]


def gpu_render(scene, cam, W, H, K, le, ld, opts=None, engine=rcp.RCP_ENGINE_CHAIN):
    s = rcp.Scene(scene, opts)
    s.set_engine(engine)
    imgs, ids = s.render(cam, W, H, K, le, ld)
    torch.cuda.synchronize()
    out = imgs.cpu().numpy(), ids.cpu().numpy()
    s.close()
    return out


AXIS_CAM = scenegen.camera_look_at([0, 0, -3], [0, 0, 0], [0, 1, 0], 60.0)
PATCH_CAM = scenegen.camera_look_at([0, 0.5, -1.4], [0, 0.05, 0], [0, 1, 0], 60.0)
OBLIQUE_CAM = scenegen.camera_look_at([1.3, -0.7, 1.9], [0.05, 0.1, -0.1], [0.2, 1, 0.1], 75.0)


# ---------------------------------------------------------------------------
# Ray generation (Section 2 ray, Section 3 colour mapping): bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cam,W,H,le,ld,seed", [
    (AXIS_CAM, 64, 64, 0.0, 0.02, 0),
    (PATCH_CAM, 67, 45, 0.01, 0.05, 1),
    (OBLIQUE_CAM, 31, 17, 0.3, 0.9, 2),
    (AXIS_CAM, 1, 1, 0.0, 0.5, 3),
    (PATCH_CAM, 1920, 1080, 0.0, 0.01, 4),
])
def test_generate_rays_bit_exact(cam, W, H, le, ld, seed):
    say("generate_rays", W, H, le, ld)
    rng = np.random.default_rng(seed)
    prev = rng.uniform(0, 1, size=(H, W, 3)).astype(np.float32)
    prev.reshape(-1, 3)[::5] = 0.5            # some seed-coloured pixels
    prev.reshape(-1, 3)[1::7] = [1.0, 0.0, 1.0]
    tp = torch.from_numpy(prev).cuda()
    org = torch.empty((H, W, 3), device="cuda")
    dirs = torch.empty((H, W, 3), device="cuda")
    rcp.rcp_generate_rays(cam, W, H, rcp.make_displacement(le, ld), tp, org, dirs)
    torch.cuda.synchronize()
    g_o = org.cpu().numpy().reshape(-1, 3)
    g_d = dirs.cpu().numpy().reshape(-1, 3)
    P = W * H
    pix = np.arange(P) if P <= 5000 else rng.choice(P, size=5000, replace=False)
    for p in pix:
        y, x = divmod(int(p), W)
        o, d = oracle.ray(cam, W, H, x, y, prev[y, x], le, ld)
        assert np.array_equal(g_o[p], o) and np.array_equal(g_d[p], d), (x, y)
    # NULL previous image = the grey seed = the undisplaced pinhole rays
    rcp.rcp_generate_rays(cam, W, H, rcp.make_displacement(le, ld), None, org, dirs)
    torch.cuda.synchronize()
    g_d = dirs.cpu().numpy().reshape(-1, 3)
    for p in pix[:200]:
        y, x = divmod(int(p), W)
        _, d = oracle.ray(cam, W, H, x, y, [0.5, 0.5, 0.5], 0.0, 0.0)
        assert np.array_equal(g_d[p], d)


# ---------------------------------------------------------------------------
# Closest hit (BVH traversal + watertight test) against oracle brute force
# ---------------------------------------------------------------------------

def _random_rays(scene, n, seed):
    rng = np.random.default_rng(seed)
    lo = scene.verts.min(0)
    hi = scene.verts.max(0)
    ctr = (lo + hi) / 2
    ext = float(np.max(hi - lo))
    o = (ctr + rng.uniform(-1.5, 1.5, size=(n, 3)) * ext).astype(np.float32)
    o[::9] = (ctr + rng.uniform(-0.3, 0.3, size=(len(o[::9]), 3)) * ext)     # origins inside the scene
    tg = ctr + rng.uniform(-0.5, 0.5, size=(n, 3)) * ext
    d = tg - o
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    for a in range(3):                           # axis-aligned rays, both signs on every axis
        d[a::11] = 0.0
        d[a::22, a] = 1.0
        d[a + 11::22, a] = -1.0
    d[5::13] *= 3.0                                                         # unnormalised directions
    return o, d


@pytest.mark.parametrize("name,scene_fn", [
    ("soup256", lambda: scenegen.soup_scene(0, 256)),
    ("soup1500", lambda: scenegen.soup_scene(3, 1500)),
    ("patch", lambda: scenegen.terrain_patch(11, 24, 8)),
    ("adversarial", lambda: scenegen.adversarial_scene()),
    ("quad", lambda: scenegen.quad_scene()),
    ("one_triangle", lambda: scenegen.soup_scene(4, 1)),
    ("two_triangles", lambda: scenegen.soup_scene(4, 2)),
    ("five_triangles", lambda: scenegen.soup_scene(4, 5)),
])
def test_trace_rays_equal_bruteforce(name, scene_fn):
    say("trace_rays", name)
    sc = scene_fn()
    n = 6000
    o, d = _random_rays(sc, n, 1)
    s = rcp.Scene(sc)
    t = torch.empty(n, device="cuda")
    i = torch.empty(n, dtype=torch.int32, device="cuda")
    f = torch.empty(n, dtype=torch.int32, device="cuda")
    rcp.rcp_trace_rays(s.handle, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), n, t, i, f)
    torch.cuda.synchronize()
    gt, gi, gf = t.cpu().numpy(), i.cpu().numpy(), f.cpu().numpy()
    ob = oracle.OracleScene(sc, use_bvh=False)
    n_hit = 0
    for r in range(n):
        hit, tt, tid, fr = ob.closest_hit(o[r], d[r], brute=True)
        if hit:
            n_hit += 1
            assert gi[r] == tid and gt[r] == np.float32(tt) and gf[r] == int(fr), (r, gi[r], tid, gt[r], tt)
        else:
            assert gi[r] == -1 and np.isinf(gt[r]), r
    assert n_hit > 0
    s.close()


def test_trace_rays_empty_scene_and_zero_rays():
    say("trace_rays empty")
    s = rcp.Scene(scenegen.empty_scene())
    assert s.info()["n_nodes"] == 0
    n = 100
    o, d = _random_rays(scenegen.soup_scene(0, 8), n, 2)
    t = torch.empty(n, device="cuda")
    i = torch.empty(n, dtype=torch.int32, device="cuda")
    rcp.rcp_trace_rays(s.handle, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), n, t, i)
    rcp.rcp_trace_rays(s.handle, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), 0, t, i)
    torch.cuda.synchronize()
    assert (i.cpu().numpy() == -1).all() and np.isinf(t.cpu().numpy()).all()
    s.close()


# ---------------------------------------------------------------------------
# K-pass renders against the oracle's K-pass loop
# ---------------------------------------------------------------------------

RENDER_CASES = [
    # name, scene factory, camera, W, H, K, lambda_eye, lambda_dir
    ("soup256", lambda: scenegen.soup_scene(0, 256), AXIS_CAM, 64, 64, 6, 0.0, 0.02),
    ("soup256_literal_eye", lambda: scenegen.soup_scene(0, 256), AXIS_CAM, 64, 64, 6, 0.02, 0.02),
    ("patch_ragged", lambda: scenegen.terrain_patch(11, 24, 8), PATCH_CAM, 67, 45, 4, 0.0, 0.05),
    ("patch_big_lambda", lambda: scenegen.terrain_patch(12, 40, 20), PATCH_CAM, 96, 72, 8, 0.05, 0.3),
    ("adversarial", lambda: scenegen.adversarial_scene(), AXIS_CAM, 50, 41, 6, 0.0, 0.1),
    ("halfplane", lambda: scenegen.halfplane_scene(), AXIS_CAM, 33, 21, 5, 0.0, 0.2),
    ("oblique_soup", lambda: scenegen.soup_scene(9, 1500), OBLIQUE_CAM, 80, 48, 6, 0.01, 0.05),
    ("lambda_zero", lambda: scenegen.terrain_patch(11, 24, 8), PATCH_CAM, 40, 30, 3, 0.0, 0.0),
    ("one_pixel", lambda: scenegen.soup_scene(0, 256), AXIS_CAM, 1, 1, 6, 0.0, 0.02),
    ("one_row", lambda: scenegen.terrain_patch(11, 24, 8), PATCH_CAM, 130, 1, 3, 0.0, 0.05),
    ("one_column", lambda: scenegen.terrain_patch(11, 24, 8), PATCH_CAM, 1, 77, 3, 0.0, 0.05),
    ("single_pass", lambda: scenegen.soup_scene(0, 256), AXIS_CAM, 64, 64, 1, 0.0, 0.02),
    ("empty_scene", lambda: scenegen.empty_scene(), AXIS_CAM, 23, 19, 4, 0.0, 0.02),
    ("one_triangle", lambda: scenegen.soup_scene(7, 1, extent=1.2), AXIS_CAM, 40, 40, 4, 0.0, 0.1),
    ("many_passes", lambda: scenegen.soup_scene(2, 300), AXIS_CAM, 48, 40, 20, 0.0, 0.05),
    # the largest pass count; 427 of the 851 pixels still change at pass 63
    ("max_passes", lambda: scenegen.terrain_patch(12, 40, 20), PATCH_CAM, 37, 23, 64, 0.0, 0.3),
    # views of 16 or more tiles a side take their work in super-tiles of
    # 16 x 16 tiles, padded at the right and bottom edges
    ("supertiles_padded", lambda: scenegen.terrain_patch(11, 24, 8), PATCH_CAM, 200, 150, 4, 0.0, 0.05),
    ("supertiles_exact", lambda: scenegen.terrain_patch(12, 40, 20), PATCH_CAM, 256, 128, 3, 0.0, 0.05),
    ("supertiles_edges", lambda: scenegen.soup_scene(9, 1500), OBLIQUE_CAM, 129, 257, 3, 0.01, 0.05),
]


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
@pytest.mark.parametrize("case", RENDER_CASES, ids=[c[0] for c in RENDER_CASES])
def test_render_matches_oracle(case, engine):
    name, scene_fn, cam, W, H, K, le, ld = case
    say("render", name, W, H, K, le, ld, "engine", engine)
    sc = scene_fn()
    g_img, g_ids = gpu_render(sc, cam, W, H, K, le, ld, engine=engine)
    o_img, o_ids = oracle.OracleScene(sc, use_bvh=True).render(cam, W, H, K, le, ld)
    r = assert_parity(g_img, g_ids, o_img, o_ids, name)
    # the path is designed to reproduce the oracle's FP32 arithmetic exactly
    assert r["exact_images"] and r["exact_ids"], r


@pytest.mark.parametrize("opts", [
    dict(max_leaf=1), dict(max_leaf=2), dict(max_leaf=8), dict(max_leaf=3, c_isect=2.0),
    dict(max_leaf=4, c_trav=3.0, c_isect=0.5), dict(builder=1), dict(builder=1, max_leaf=1),
    dict(collapse=1), dict(collapse=1, builder=1, max_leaf=2), dict(collapse=0, c_trav=4.0, max_leaf=8),
])
def test_build_options_do_not_change_the_image(opts):
    say("build options", opts)
    sc = scenegen.terrain_patch(12, 40, 20)
    base = gpu_render(sc, PATCH_CAM, 57, 43, 4, 0.0, 0.05)
    other = gpu_render(sc, PATCH_CAM, 57, 43, 4, 0.0, 0.05, rcp.build_options(**opts))
    assert np.array_equal(base[0], other[0]) and np.array_equal(base[1], other[1])


@pytest.mark.parametrize("W,H", [(61, 47), (200, 150)])
def test_render_pass_chain_equals_render(W, H):
    """rcp_render_pass applied to image k-1 gives image k (each pass starts
    from the base camera; only the image carries state)."""
    say("render_pass chain", W, H)
    sc = scenegen.terrain_patch(11, 24, 8)
    K = 5
    s = rcp.Scene(sc)
    imgs, ids = s.render(PATCH_CAM, W, H, K, 0.01, 0.05)
    d = rcp.make_displacement(0.01, 0.05)
    prev = None
    for k in range(K):
        out = torch.empty((H, W, 3), device="cuda")
        oid = torch.empty((H, W), dtype=torch.int32, device="cuda")
        rcp.rcp_render_pass(s.handle, PATCH_CAM, W, H, d, prev, out, oid)
        torch.cuda.synchronize()
        assert torch.equal(out, imgs[k]) and torch.equal(oid, ids[k]), k
        prev = out
    s.close()


def test_render_pass_pointwise():
    """Perturbing one pixel of the previous image changes that pixel only."""
    say("render_pass pointwise")
    sc = scenegen.terrain_patch(11, 24, 8)
    W, H = 40, 30
    s = rcp.Scene(sc)
    imgs, _ = s.render(PATCH_CAM, W, H, 1, 0.0, 0.05)
    d = rcp.make_displacement(0.0, 0.05)
    base = torch.empty((H, W, 3), device="cuda")
    rcp.rcp_render_pass(s.handle, PATCH_CAM, W, H, d, imgs[0].contiguous(), base, None)
    rng = np.random.default_rng(0)
    for _ in range(5):
        y, x = int(rng.integers(0, H)), int(rng.integers(0, W))
        p2 = imgs[0].clone()
        p2[y, x] = torch.tensor(rng.uniform(0, 1, 3), dtype=torch.float32)
        out = torch.empty_like(base)
        rcp.rcp_render_pass(s.handle, PATCH_CAM, W, H, d, p2, out, None)
        torch.cuda.synchronize()
        diff = (out != base).any(-1).cpu().numpy()
        diff[y, x] = False
        assert not diff.any()
    s.close()


def test_prefix_stability_and_determinism():
    say("prefix stability")
    sc = scenegen.soup_scene(2, 300)
    a = gpu_render(sc, AXIS_CAM, 48, 40, 8, 0.0, 0.05)
    b = gpu_render(sc, AXIS_CAM, 48, 40, 3, 0.0, 0.05)
    c = gpu_render(sc, AXIS_CAM, 48, 40, 8, 0.0, 0.05)
    assert np.array_equal(a[0][:3], b[0]) and np.array_equal(a[1][:3], b[1])
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
def test_stats_kernel_counts_and_images(engine):
    say("render_stats engine", engine)
    w = scenegen.workload("soup256")
    s = rcp.Scene(w.scene)
    imgs, ids = s.render(w.camera, 64, 64, 6, 0.0, 0.02)
    s.set_engine(engine)
    i2 = torch.empty_like(imgs)
    d2 = torch.empty_like(ids)
    counts = rcp.rcp_render_stats(s.handle, w.camera, 64, 64, 6, rcp.make_displacement(0.0, 0.02), i2, d2)
    assert torch.equal(imgs, i2) and torch.equal(ids, d2)
    assert np.all(counts[:, 1] > 0) == np.all(counts[:, 0] > 0) and np.all(counts[:, 2] >= 0)
    assert counts[0, 0] == 64 * 64
    for k in range(5):
        assert counts[k + 1, 0] == counts[k, 3]          # traced at k+1 = appended at k
    # appended at pass 0 = pixels whose first colour differs from the grey seed
    im = imgs.cpu().numpy()
    assert counts[0, 3] == int(np.sum(np.any(im[0] != np.float32(0.5), axis=-1)))
    assert counts[5, 3] == 0
    s.close()


# ---------------------------------------------------------------------------
# The largest image (whole-frame checks of the full-size workloads are in
# test_gpu_wholeframe.py)
# ---------------------------------------------------------------------------

def test_maximum_image_size():
    """W * H = 2^27 (the limit) on a small scene; sampled chains."""
    sc = scenegen.soup_scene(0, 256)
    cam = AXIS_CAM
    W, H, K = 16384, 8192, 2
    say("maximum size", W, H, K)
    s = rcp.Scene(sc)
    imgs = torch.empty((K, H, W, 3), device="cuda")
    rcp.rcp_render(s.handle, cam, W, H, K, rcp.make_displacement(0.0, 0.02), imgs, None)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    P = W * H
    pix = rng.choice(P, size=3000, replace=False)
    g = imgs.reshape(K, P, 3)[:, torch.from_numpy(pix).cuda()].permute(1, 0, 2).cpu().numpy()
    o_img, _ = oracle.OracleScene(sc, use_bvh=True).render_pixels(cam, W, H, K, 0.0, 0.02, pix.astype(np.int32))
    assert np.array_equal(g, o_img)
    del imgs
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render(s.handle, cam, W, H + 1, 1, rcp.make_displacement(0.0, 0.02), 1, None)
    s.close()


def test_invalid_arguments_with_a_real_scene():
    say("invalid arguments")
    w = scenegen.workload("soup256")
    s = rcp.Scene(w.scene)
    out = torch.empty((2, 8, 8, 3), device="cuda")
    d = rcp.make_displacement(0.0, 0.02)
    for K in (0, 65):
        with pytest.raises(rcp.RcpError) as e:
            rcp.rcp_render(s.handle, w.camera, 8, 8, K, d, out)
        assert e.value.status == rcp.RCP_ERR_INVALID_ARGUMENT
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render(s.handle, w.camera, 8, 8, 2, rcp.make_displacement(0.0, 1.5), out)
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render(s.handle, w.camera, 8, 8, 2, d, None)
    s.close()


def test_engines_trace_the_same_rays():
    """Both engines trace exactly the pixels whose inputs changed, pass by
    pass; node and triangle counts may differ slightly, since speculative
    traversal depends on which rays share a wave."""
    w = scenegen.workload("terrain1m")
    say("engines stats", w.name)
    s = rcp.Scene(w.scene)
    d = rcp.make_displacement(w.lambda_eye, w.lambda_dir)
    out = {}
    for e in ENGINES:
        s.set_engine(e)
        img = torch.empty((w.passes, w.height, w.width, 3), device="cuda")
        out[e] = (rcp.rcp_render_stats(s.handle, w.camera, w.width, w.height, w.passes, d, img, None), img)
    (c0, i0), (c1, i1) = out[ENGINES[0]], out[ENGINES[1]]
    assert torch.equal(i0, i1)
    assert np.array_equal(c0[:, 0], c1[:, 0]) and np.array_equal(c0[:, 3], c1[:, 3])
    assert c0[0, 0] == w.width * w.height
    for col in (1, 2):
        a, b = c0[:, col].astype(np.float64), c1[:, col].astype(np.float64)
        assert np.all(np.abs(a - b) <= 0.05 * np.maximum(a, b) + 64), (col, a, b)
    s.close()
