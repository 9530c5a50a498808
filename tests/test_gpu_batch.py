"""Batched rendering, HIP-graph replays and launch tuning.

Every view of a batch must equal rcp_render of that view alone (both are
bit-exact against the oracle, which is checked on a sample); graph replays
must equal the eager render, also with eager work between replays; tuning
parameters change the speed only, never an image."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_2312_12392_amd import rcp

pytestmark = pytest.mark.gpu

PATCH_CAM = scenegen.camera_look_at([0, 0.5, -1.4], [0, 0.05, 0], [0, 1, 0], 60.0)


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    rcp.load()


def single(s, cam, W, H, K, le, ld):
    imgs, ids = s.render(cam, W, H, K, le, ld)
    torch.cuda.synchronize()
    return imgs, ids


def test_batch_equals_single_views_and_oracle():
    sc = scenegen.terrain_patch(12, 40, 20)
    s = rcp.Scene(sc)
    rng = np.random.default_rng(0)
    specs = []
    for i, (W, H, K) in enumerate([(67, 45, 4), (1, 1, 6), (130, 1, 3), (1, 77, 2), (64, 64, 8), (33, 21, 1),
                                   (96, 72, 5), (40, 30, 7), (8, 8, 3), (57, 43, 6), (128, 96, 2), (20, 50, 4)]):
        ang = rng.uniform(-0.6, 0.6)
        cam = scenegen.camera_look_at([1.4 * np.sin(ang), rng.uniform(0.3, 0.7), -1.4 * np.cos(ang)],
                                      [0, 0.05, 0], [0, 1, 0], float(rng.uniform(40, 80)))
        le = 0.02 if i % 3 == 0 else 0.0
        ld = float(rng.uniform(0.0, 0.2))
        specs.append((cam, W, H, K, le, ld))
    say("batch of", len(specs), "views")
    outs = [(torch.full((K, H, W, 3), -1.0, device="cuda"), torch.full((K, H, W), -7, dtype=torch.int32, device="cuda"))
            for (_, W, H, K, _, _) in specs]
    views = [(cam, W, H, K, rcp.make_displacement(le, ld), o, i) for (cam, W, H, K, le, ld), (o, i) in zip(specs, outs)]
    rcp.rcp_render_batch(s.handle, views)
    torch.cuda.synchronize()
    orc = oracle.OracleScene(sc, use_bvh=True)
    for n, ((cam, W, H, K, le, ld), (o, i)) in enumerate(zip(specs, outs)):
        ref_img, ref_ids = single(s, cam, W, H, K, le, ld)
        assert torch.equal(o, ref_img) and torch.equal(i, ref_ids), n
        if n % 3 == 0:
            oi, oid = orc.render(cam, W, H, K, le, ld)
            assert np.array_equal(o.cpu().numpy(), oi) and np.array_equal(i.cpu().numpy(), oid), n
    s.close()


def test_batch_mixed_modes_equal_single_views_and_oracle():
    """Colour, depth and normal views in one call: one launch per mode, each
    view equal to rcp_render alone and to the oracle."""
    sc = scenegen.terrain_patch(12, 40, 20)
    s = rcp.Scene(sc)
    orc = oracle.OracleScene(sc, use_bvh=True)
    rng = np.random.default_rng(5)
    modes = [rcp.RCP_MODE_DEPTH, rcp.RCP_MODE_COLOR, rcp.RCP_MODE_NORMAL, rcp.RCP_MODE_NORMAL, rcp.RCP_MODE_COLOR,
             rcp.RCP_MODE_DEPTH, rcp.RCP_MODE_DEPTH, rcp.RCP_MODE_COLOR]
    specs = []
    for i, mode in enumerate(modes):
        ang = rng.uniform(-0.6, 0.6)
        cam = scenegen.camera_look_at([1.4 * np.sin(ang), rng.uniform(0.3, 0.7), -1.4 * np.cos(ang)],
                                      [0, 0.05, 0], [0, 1, 0], 60.0)
        W, H, K = [(67, 45, 4), (1, 1, 3), (40, 30, 6), (96, 72, 2), (33, 21, 5), (64, 64, 6), (8, 3, 2),
                   (50, 41, 7)][i]
        specs.append((cam, W, H, K, 0.01 * (i % 2), float(rng.uniform(0.02, 0.2)), mode, float(rng.uniform(0.5, 2))))
    say("mixed-mode batch", len(specs))
    outs = [(torch.empty((K, H, W, 3), device="cuda"), torch.empty((K, H, W), dtype=torch.int32, device="cuda"))
            for (_, W, H, K, *_r) in specs]
    rcp.rcp_render_batch(s.handle, [(cam, W, H, K, rcp.make_displacement(le, ld, mode, z0), o, i)
                                    for (cam, W, H, K, le, ld, mode, z0), (o, i) in zip(specs, outs)])
    torch.cuda.synchronize()
    for n, ((cam, W, H, K, le, ld, mode, z0), (o, i)) in enumerate(zip(specs, outs)):
        ref_img, ref_ids = s.render(cam, W, H, K, le, ld, mode=mode, z0=z0)
        torch.cuda.synchronize()
        assert torch.equal(o, ref_img) and torch.equal(i, ref_ids), n
        oi, oid = orc.render(cam, W, H, K, le, ld, mode=mode, z0=z0)
        assert np.array_equal(o.cpu().numpy(), oi) and np.array_equal(i.cpu().numpy(), oid), n
    s.close()


def test_batch_orbit_mix_on_terrain1m():
    """The 64-view orbit mix (256^2 .. 1024^2, K 1..8) of the 1M scene: every
    view equals rcp_render of that view alone (the oracle checks every pixel
    of every view in test_gpu_wholeframe.py)."""
    w = scenegen.workload("terrain1m")
    views = scenegen.orbit_views(3, 64)
    say("orbit mix", len(views))
    s = rcp.Scene(w.scene)
    d = rcp.make_displacement(0.0, 0.01)
    outs = [torch.empty((K, H, W, 3), device="cuda") for (_, W, H, K) in views]
    rcp.rcp_render_batch(s.handle, [(cam, W, H, K, d, o, None) for (cam, W, H, K), o in zip(views, outs)])
    torch.cuda.synchronize()
    for n, ((cam, W, H, K), o) in enumerate(zip(views, outs)):
        ref, _ = single(s, cam, W, H, K, 0.0, 0.01)
        assert torch.equal(o, ref), n
    s.close()


def test_batch_of_the_maximum_view_count():
    """1024 views (the limit) of mixed tiny sizes, K 1..6 and all three
    modes in one call: each equals its single render, every 32nd the oracle;
    1025 views are rejected."""
    sc = scenegen.terrain_patch(11, 24, 8)
    s = rcp.Scene(sc)
    rng = np.random.default_rng(11)
    specs = []
    for i in range(1024):
        ang = rng.uniform(-0.7, 0.7)
        cam = scenegen.camera_look_at([1.4 * np.sin(ang), rng.uniform(0.3, 0.7), -1.4 * np.cos(ang)],
                                      [0, 0.05, 0], [0, 1, 0], 60.0)
        W, H, K = int(rng.integers(1, 13)), int(rng.integers(1, 13)), int(rng.integers(1, 7))
        d = rcp.make_displacement(0.0, float(rng.uniform(0.0, 0.1)), mode=i % 3, z0=1.2)
        specs.append((cam, W, H, K, d))
    outs = [(torch.full((K, H, W, 3), -1.0, device="cuda"), torch.full((K, H, W), -7, dtype=torch.int32, device="cuda"))
            for (_, W, H, K, _) in specs]
    say("batch of 1024 views")
    rcp.rcp_render_batch(s.handle, [(cam, W, H, K, d, o, i) for (cam, W, H, K, d), (o, i) in zip(specs, outs)])
    torch.cuda.synchronize()
    orc = oracle.OracleScene(sc, use_bvh=True)
    for n, ((cam, W, H, K, d), (o, i)) in enumerate(zip(specs, outs)):
        ref_o = torch.empty_like(o)
        ref_i = torch.empty_like(i)
        rcp.rcp_render(s.handle, cam, W, H, K, d, ref_o, ref_i)
        torch.cuda.synchronize()
        assert torch.equal(o, ref_o) and torch.equal(i, ref_i), n
        if n % 32 == 0:
            oi, oid = orc.render(cam, W, H, K, d.lambda_eye, d.lambda_dir, mode=d.mode, z0=d.z0)
            assert np.array_equal(o.cpu().numpy(), oi) and np.array_equal(i.cpu().numpy(), oid), n
    orc.close()
    extra = torch.empty((1, 1, 1, 3), device="cuda")
    views = [(cam, W, H, K, d, o, None) for (cam, W, H, K, d), (o, _) in zip(specs, outs)]
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render_batch(s.handle, views + [(specs[0][0], 1, 1, 1, specs[0][4], extra, None)])
    s.close()


def test_one_view_batch_is_a_single_render():
    """A batch of one view hands its tiles out in cost order, as rcp_render
    does (and in screen order with tile_order 0): the same images either way."""
    sc = scenegen.terrain_patch(14, 40, 20)
    s = rcp.Scene(sc)
    for W, H, K in [(67, 45, 5), (1, 1, 3), (200, 9, 6), (128, 128, 2)]:
        ref_img, ref_ids = single(s, PATCH_CAM, W, H, K, 0.0, 0.07)
        for order in (1, 0):
            say("one-view batch", W, H, K, "tile_order", order)
            rcp.rcp_set_tuning(s.handle, tile_order=order)
            o = torch.full((K, H, W, 3), -1.0, device="cuda")
            i = torch.full((K, H, W), -7, dtype=torch.int32, device="cuda")
            rcp.rcp_render_batch(s.handle, [(PATCH_CAM, W, H, K, rcp.make_displacement(0.0, 0.07), o, i)])
            torch.cuda.synchronize()
            assert torch.equal(o, ref_img) and torch.equal(i, ref_ids), (W, H, K, order)
        rcp.rcp_set_tuning(s.handle, tile_order=1)
    s.close()


def test_batch_rejects_bad_views():
    w = scenegen.workload("soup256")
    s = rcp.Scene(w.scene)
    o = torch.empty((2, 8, 8, 3), device="cuda")
    d = rcp.make_displacement(0.0, 0.02)
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render_batch(s.handle, [(w.camera, 8, 8, 2, d, o, None), (w.camera, 8, 8, 2, d, o, None)])  # overlap
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render_batch(s.handle, [(w.camera, 8, 8, 0, d, o, None)])                         # K = 0
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render_batch(s.handle, [(w.camera, 8, 8, 2, rcp.make_displacement(0.0, 0.02, 7), o, None)])
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render_batch(s.handle, [])
    s.close()


@pytest.mark.parametrize("engine", [rcp.RCP_ENGINE_CHAIN, rcp.RCP_ENGINE_PASSES], ids=["chain", "passes"])
def test_graph_replays_equal_eager_render(engine):
    w = scenegen.workload("soup256")
    say("graph replays engine", engine)
    s = rcp.Scene(w.scene)
    s.set_engine(engine)
    ref_img, ref_ids = single(s, w.camera, 64, 64, 6, 0.0, 0.02)
    out = torch.empty_like(ref_img)
    ids = torch.empty_like(ref_ids)
    g = rcp.rcp_graph_create(s.handle, w.camera, 64, 64, 6, rcp.make_displacement(0.0, 0.02), out, ids)
    for r in range(4):
        out.zero_()
        ids.zero_()
        torch.cuda.synchronize()
        rcp.rcp_graph_launch(g)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_img) and torch.equal(ids, ref_ids), r
        # eager work between replays, on the same scene and stream
        single(s, w.camera, 40, 30, 3, 0.0, 0.05)
    # new camera and displacement in place
    cam2 = scenegen.camera_look_at([0.4, 0.3, -2.8], [0, 0, 0], [0, 1, 0], 55.0)
    rcp.rcp_graph_update(g, cam2, rcp.make_displacement(0.01, 0.05))
    ref2, ref2_ids = single(s, cam2, 64, 64, 6, 0.01, 0.05)
    for r in range(3):
        out.zero_()
        torch.cuda.synchronize()
        rcp.rcp_graph_launch(g)
        torch.cuda.synchronize()
        assert torch.equal(out, ref2) and torch.equal(ids, ref2_ids), r
    rcp.rcp_graph_destroy(g)
    s.close()


@pytest.mark.parametrize("tuning", [
    dict(refill_min=1, blocks_per_cu=1, tile_log2w=0, engine=0, exit_lanes=0),
    dict(refill_min=64, blocks_per_cu=2, tile_log2w=6, engine=0, exit_lanes=64),
    dict(refill_min=17, blocks_per_cu=0, tile_log2w=4, engine=1, exit_lanes=3),
    dict(refill_min=40, blocks_per_cu=3, tile_log2w=2, engine=1, exit_lanes=64),
    dict(refill_min=1, blocks_per_cu=1, tile_log2w=0, engine=1, exit_lanes=1),
    dict(refill_min=64, blocks_per_cu=0, tile_log2w=3, engine=0, exit_lanes=1),
    dict(refill_min=56, blocks_per_cu=0, tile_log2w=3, engine=0, exit_lanes=16, top_levels=0),
    dict(refill_min=56, blocks_per_cu=0, tile_log2w=3, engine=0, exit_lanes=16, top_levels=2, stack_entries=8),
    dict(refill_min=48, blocks_per_cu=0, tile_log2w=3, engine=0, exit_lanes=8, block_size=512),
    dict(refill_min=30, blocks_per_cu=2, tile_log2w=4, engine=0, exit_lanes=12, top_levels=3, stack_entries=8,
         block_size=512),
    dict(refill_min=56, blocks_per_cu=0, tile_log2w=3, engine=0, exit_lanes=16, tile_order=0),
    dict(refill_min=64, blocks_per_cu=1, tile_log2w=6, engine=0, exit_lanes=4, tile_order=0),
])
def test_tuning_does_not_change_images(tuning):
    say("tuning", tuning)
    sc = scenegen.terrain_patch(12, 40, 20)
    s = rcp.Scene(sc)
    ref_img, ref_ids = single(s, PATCH_CAM, 67, 45, 5, 0.0, 0.1)
    t = dict(top_levels=4, stack_entries=16, block_size=256, tile_order=1)
    t.update(tuning)
    rcp.rcp_set_tuning(s.handle, **t)
    assert rcp.rcp_get_tuning(s.handle) == t
    img, ids = single(s, PATCH_CAM, 67, 45, 5, 0.0, 0.1)
    assert torch.equal(img, ref_img) and torch.equal(ids, ref_ids)
    # the batch kernel follows the same parameters
    o = torch.empty_like(img)
    rcp.rcp_render_batch(s.handle, [(PATCH_CAM, 67, 45, 5, rcp.make_displacement(0.0, 0.1), o, None)])
    torch.cuda.synchronize()
    assert torch.equal(o, ref_img)
    s.close()


def test_autotune_and_cache(tmp_path):
    w = scenegen.workload("soup256")
    say("autotune")
    s = rcp.Scene(w.scene)
    ref_img, _ = single(s, w.camera, 64, 64, 6, 0.0, 0.02)
    out = torch.empty_like(ref_img)
    t, ms = rcp.rcp_autotune(s.handle, w.camera, 64, 64, 6, rcp.make_displacement(0.0, 0.02), out, None, repeats=2)
    torch.cuda.synchronize()
    assert ms > 0 and 1 <= t["refill_min"] <= 64
    assert rcp.rcp_get_tuning(s.handle) == t
    assert torch.equal(out, ref_img)
    path = str(tmp_path / "tune.json")
    t1 = rcp.autotune_cached(s.handle, "soup256", w.camera, 64, 64, 6, rcp.make_displacement(0.0, 0.02), out,
                             cache_path=path, repeats=1)
    assert os.path.exists(path) and len(json.load(open(path))) == 1
    rcp.rcp_set_tuning(s.handle, refill_min=40, blocks_per_cu=0, tile_log2w=3, top_levels=1, stack_entries=8)
    t2 = rcp.autotune_cached(s.handle, "soup256", w.camera, 64, 64, 6, rcp.make_displacement(0.0, 0.02), out,
                             cache_path=path, repeats=1)
    assert t2 == t1 and rcp.rcp_get_tuning(s.handle) == t1
    s.close()


def test_autotune_batch():
    """The autotuner on a batch picks valid parameters (the engine stays the
    chain engine) and leaves the batch's images in the outputs."""
    sc = scenegen.terrain_patch(12, 40, 20)
    s = rcp.Scene(sc)
    specs = [(PATCH_CAM, 67, 45, 4), (PATCH_CAM, 33, 21, 2), (PATCH_CAM, 96, 72, 6)]
    refs = [single(s, cam, W, H, K, 0.0, 0.05) for (cam, W, H, K) in specs]
    outs = [torch.full((K, H, W, 3), -1.0, device="cuda") for (_, W, H, K) in specs]
    d = rcp.make_displacement(0.0, 0.05)
    say("autotune batch")
    t, ms = rcp.rcp_autotune_batch(s.handle, [(cam, W, H, K, d, o, None) for (cam, W, H, K), o in zip(specs, outs)],
                                   repeats=1)
    torch.cuda.synchronize()
    assert ms > 0 and t["engine"] == rcp.RCP_ENGINE_CHAIN
    assert t["stack_entries"] in (8, 16) and t["block_size"] in (256, 512) and 0 <= t["top_levels"] <= 4
    assert rcp.rcp_get_tuning(s.handle) == t
    for o, (ref, _) in zip(outs, refs):
        assert torch.equal(o, ref)
    s.close()
