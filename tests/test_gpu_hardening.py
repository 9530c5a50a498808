"""Paths that ordinary renders rarely reach, each forced on purpose:

* the traversal stack's overflow from LDS into global memory, on a scene of
  thousands of stacked quads that every ray crosses (the spill counter must
  be non-zero, and the images equal the oracle's);
* HIP graphs replayed after the scene's own workspace grew and changed
  (larger renders, another mode, the other engine in between);
* a ray that runs out of its traversal step budget (lowered from the host
  through the test hook): the render completes, the hit is a miss, and the
  error is reported as RCP_ERR_INTERNAL;
* device allocations failing at every point of a scene build and of a
  render's first workspace allocation (test hook): RCP_ERR_OUT_OF_MEMORY,
  and the library keeps working afterwards.

No case makes the GPU fault or hang: every kernel runs to its normal end.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_2312_12392_amd import rcp

pytestmark = pytest.mark.gpu

AXIS_CAM = scenegen.camera_look_at([0, 0, -3], [0, 0, 0], [0, 1, 0], 60.0)
PATCH_CAM = scenegen.camera_look_at([0, 0.5, -1.4], [0, 0.05, 0], [0, 1, 0], 60.0)


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    rcp.load()
    yield
    rcp.rcp_debug_set(rcp.RCP_DEBUG_FAIL_ALLOC_AFTER, -1)
    rcp.rcp_debug_set(rcp.RCP_DEBUG_STEP_BUDGET, 0)


def stacked_quads(n_quads, seed=0, half=1.0, dz=0.002):
    """n_quads squares of side 2*half facing -z, one behind the other along
    the view axis (z = i * dz), each a little offset so that no two coincide,
    with random colours: every ray through the middle crosses all of them."""
    rng = np.random.default_rng(seed)
    verts, idx = [], []
    for i in range(n_quads):
        ox, oy = rng.uniform(-0.05, 0.05, 2)
        z = i * dz
        b = len(verts)
        verts += [[ox - half, oy - half, z], [ox + half, oy - half, z], [ox - half, oy + half, z],
                  [ox + half, oy + half, z]]
        idx += [[b, b + 1, b + 2], [b + 2, b + 1, b + 3]]
    rgb = rng.uniform(0, 1, size=(len(idx), 3))
    return scenegen.Scene(verts=np.asarray(verts, np.float32), idx=np.asarray(idx, np.uint32),
                          rgb=rgb.astype(np.float32), name=f"stacked{n_quads}")


def test_stack_overflow_with_the_shallow_lds_stack():
    """The chain kernel with 8 LDS stack entries (and workgroups of 512)
    spills more often; its images stay equal to the oracle's."""
    sc = stacked_quads(2048, seed=1)
    W, H, K = 40, 32, 4
    say("stacked quads, 8-entry stack")
    s = rcp.Scene(sc, rcp.build_options(max_leaf=1))
    o_img, o_ids = oracle.OracleScene(sc, use_bvh=True).render(AXIS_CAM, W, H, K, 0.0, 0.05)
    for stack, block in [(8, 256), (8, 512), (16, 512)]:
        rcp.rcp_set_tuning(s.handle, stack_entries=stack, block_size=block)
        img, ids = s.render(AXIS_CAM, W, H, K, 0.0, 0.05)
        torch.cuda.synchronize()
        assert np.array_equal(img.cpu().numpy(), o_img) and np.array_equal(ids.cpu().numpy(), o_ids), (stack, block)
        # and through the batch kernel
        o = torch.empty_like(img)
        rcp.rcp_render_batch(s.handle, [(AXIS_CAM, W, H, K, rcp.make_displacement(0.0, 0.05), o, None),
                                        (AXIS_CAM, 9, 7, 2, rcp.make_displacement(0.0, 0.05), torch.empty(
                                            (2, 7, 9, 3), device="cuda"), None)])
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy(), o_img), (stack, block)
    s.close()


@pytest.mark.parametrize("engine", [rcp.RCP_ENGINE_CHAIN, rcp.RCP_ENGINE_PASSES], ids=["chain", "passes"])
def test_stack_overflow_path_is_reached_and_exact(engine):
    sc = stacked_quads(4096)
    W, H, K, le, ld = 48, 40, 3, 0.0, 0.05
    say("stacked quads", sc.n_tris, "engine", engine)
    s = rcp.Scene(sc, rcp.build_options(max_leaf=1))
    s.set_engine(engine)
    img = torch.empty((K, H, W, 3), device="cuda")
    ids = torch.empty((K, H, W), dtype=torch.int32, device="cuda")
    counts = rcp.rcp_render_stats(s.handle, AXIS_CAM, W, H, K, rcp.make_displacement(le, ld), img, ids)
    spilled = int(counts[:, 5].sum())
    assert spilled > 0, counts
    o_img, o_ids = oracle.OracleScene(sc, use_bvh=True).render(AXIS_CAM, W, H, K, le, ld)
    assert np.array_equal(img.cpu().numpy(), o_img) and np.array_equal(ids.cpu().numpy(), o_ids)
    # the timed kernel (no counters) gives the same images
    i2, d2 = s.render(AXIS_CAM, W, H, K, le, ld)
    torch.cuda.synchronize()
    assert torch.equal(i2, img) and torch.equal(d2, ids)
    s.close()


def test_lds_counter_counts_staged_levels_only():
    """The chain engine reads the top levels of the tree from LDS; the
    per-pass engine stages nothing, so its LDS count is zero."""
    w = scenegen.workload("soup256")
    s = rcp.Scene(w.scene)
    d = rcp.make_displacement(0.0, 0.02)
    img = torch.empty((6, 64, 64, 3), device="cuda")
    c_chain = rcp.rcp_render_stats(s.handle, w.camera, 64, 64, 6, d, img, None)
    s.set_engine(rcp.RCP_ENGINE_PASSES)
    c_pass = rcp.rcp_render_stats(s.handle, w.camera, 64, 64, 6, d, img, None)
    assert c_chain[:, 4].sum() > 0 and np.all(c_chain[:, 4] <= c_chain[:, 1])
    assert c_pass[:, 4].sum() == 0
    s.close()


@pytest.mark.parametrize("engine", [rcp.RCP_ENGINE_CHAIN, rcp.RCP_ENGINE_PASSES], ids=["chain", "passes"])
def test_graph_survives_workspace_growth(engine):
    """A graph owns its buffers: renders that make the scene's workspace
    grow (larger images, more passes, another mode, the other engine)
    between replays leave every replay equal to an eager render."""
    sc = scenegen.terrain_patch(12, 40, 20)
    s = rcp.Scene(sc)
    s.set_engine(engine)
    W, H, K = 40, 30, 4
    d = rcp.make_displacement(0.0, 0.05)
    out = torch.empty((K, H, W, 3), device="cuda")
    ids = torch.empty((K, H, W), dtype=torch.int32, device="cuda")
    say("graph growth engine", engine)
    g = rcp.rcp_graph_create(s.handle, PATCH_CAM, W, H, K, d, out, ids)
    ref_img, ref_ids = s.render(PATCH_CAM, W, H, K, 0.0, 0.05)
    torch.cuda.synchronize()
    other = [(257, 193, 6, rcp.RCP_MODE_COLOR), (300, 220, 8, rcp.RCP_MODE_DEPTH),
             (320, 240, 5, rcp.RCP_MODE_NORMAL)]
    for rep, (W2, H2, K2, mode) in enumerate(other):
        out.fill_(-1.0)
        ids.fill_(-7)
        big = torch.empty((K2, H2, W2, 3), device="cuda")
        rcp.rcp_render(s.handle, PATCH_CAM, W2, H2, K2, rcp.make_displacement(0.0, 0.05, mode, 1.0), big, None)
        s.set_engine(rcp.RCP_ENGINE_PASSES if rep % 2 == 0 else rcp.RCP_ENGINE_CHAIN)
        big2 = torch.empty((K2, H2 + 5, W2 + 3, 3), device="cuda")
        rcp.rcp_render(s.handle, PATCH_CAM, W2 + 3, H2 + 5, K2, rcp.make_displacement(0.0, 0.05, mode, 1.0), big2,
                       None)
        rcp.rcp_graph_launch(g)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_img) and torch.equal(ids, ref_ids), rep
        del big, big2
    rcp.rcp_graph_destroy(g)
    s.close()


def test_step_budget_exhaustion_is_reported():
    sc = scenegen.terrain_patch(12, 40, 20)
    W, H, K = 40, 30, 3
    d = rcp.make_displacement(0.0, 0.05)
    rcp.rcp_debug_set(rcp.RCP_DEBUG_STEP_BUDGET, 2)
    try:
        s = rcp.Scene(sc)
    finally:
        rcp.rcp_debug_set(rcp.RCP_DEBUG_STEP_BUDGET, 0)
    say("step budget 2")
    img = torch.empty((K, H, W, 3), device="cuda")
    rcp.rcp_render(s.handle, PATCH_CAM, W, H, K, d, img, None)
    with pytest.raises(rcp.RcpError) as e:
        rcp.rcp_check(s.handle)
    assert e.value.status == rcp.RCP_ERR_INTERNAL and "step budget" in str(e.value)
    rcp.rcp_check(s.handle)                       # reported once, then cleared
    with pytest.raises(rcp.RcpError) as e:
        rcp.rcp_render_stats(s.handle, PATCH_CAM, W, H, K, d, img, None)
    assert e.value.status == rcp.RCP_ERR_INTERNAL
    s.set_engine(rcp.RCP_ENGINE_PASSES)
    rcp.rcp_render(s.handle, PATCH_CAM, W, H, K, d, img, None)
    with pytest.raises(rcp.RcpError):
        rcp.rcp_check(s.handle)
    s.close()
    # a scene built with the default budget renders without the error
    s = rcp.Scene(sc)
    imgs, _ = s.render(PATCH_CAM, W, H, K, 0.0, 0.05)
    rcp.rcp_check(s.handle)
    o, _ = oracle.OracleScene(sc, use_bvh=True).render(PATCH_CAM, W, H, K, 0.0, 0.05)
    assert np.array_equal(imgs.cpu().numpy(), o)
    s.close()


@pytest.mark.parametrize("mode", [rcp.RCP_MODE_COLOR, rcp.RCP_MODE_DEPTH], ids=["colour", "depth"])
def test_list_canary_mode(mode):
    """The per-pass engine's lists of continuing pixels, canary-filled before
    each pass and checked after it: clean renders pass the check with
    unchanged images; a check told that each list is one entry shorter
    reports the last entry as written past the end."""
    sc = scenegen.terrain_patch(12, 40, 20)
    W, H, K = 61, 47, 5
    d = rcp.make_displacement(0.0, 0.05, mode=mode, z0=1.2)
    s = rcp.Scene(sc)
    s.set_engine(rcp.RCP_ENGINE_PASSES)
    ref = torch.empty((K, H, W, 3), device="cuda")
    rcp.rcp_render(s.handle, PATCH_CAM, W, H, K, d, ref, None)
    counts = rcp.rcp_render_stats(s.handle, PATCH_CAM, W, H, K, d, torch.empty_like(ref), None)
    assert counts[0, 3] > 0                        # the first list is not empty
    img = torch.empty_like(ref)
    try:
        say("list canary on, mode", mode)
        rcp.rcp_debug_set(rcp.RCP_DEBUG_LIST_CANARY, 1)
        rcp.rcp_render(s.handle, PATCH_CAM, W, H, K, d, img, None)
        rcp.rcp_check(s.handle)
        assert torch.equal(img, ref)
        say("list canary with the count shortened by one")
        rcp.rcp_debug_set(rcp.RCP_DEBUG_LIST_CANARY, 2)
        rcp.rcp_render(s.handle, PATCH_CAM, W, H, K, d, img, None)
        with pytest.raises(rcp.RcpError) as e:
            rcp.rcp_check(s.handle)
        assert e.value.status == rcp.RCP_ERR_INTERNAL and "canary" in str(e.value)
        assert torch.equal(img, ref)                # the check reads only
    finally:
        rcp.rcp_debug_set(rcp.RCP_DEBUG_LIST_CANARY, 0)
    rcp.rcp_render(s.handle, PATCH_CAM, W, H, K, d, img, None)
    rcp.rcp_check(s.handle)
    s.close()


def test_build_log_line_and_leaf_histogram(capfd, monkeypatch):
    """RCP_LOG=1 prints the build statistics; the leaf histogram sums to the
    leaf count and, weighted by leaf size, to the triangle count."""
    sc = scenegen.terrain_patch(12, 40, 20)
    monkeypatch.setenv("RCP_LOG", "1")
    for ml in (1, 3, 8):
        s = rcp.Scene(sc, rcp.build_options(max_leaf=ml))
        info = s.info()
        s.close()
        h = info["leaf_hist"]
        assert sum(h) == info["n_leaves"]
        assert sum((c + 1) * n for c, n in enumerate(h)) == sc.n_tris
        assert all(n == 0 for n in h[ml:])
        err = capfd.readouterr().err
        line = [ln for ln in err.splitlines() if ln.startswith("rcp: scene built:")]
        assert len(line) == 1, err
        assert f"{sc.n_tris} triangles, {info['n_nodes']} nodes, {info['n_leaves']} leaves" in line[0]
        assert line[0].endswith(" ".join(str(n) for n in h))
    monkeypatch.delenv("RCP_LOG")
    s = rcp.Scene(sc)
    s.close()
    assert "rcp: scene built" not in capfd.readouterr().err


def test_allocation_failures_everywhere():
    sc = scenegen.terrain_patch(11, 24, 8)
    W, H, K = 40, 30, 3
    o_img, o_ids = oracle.OracleScene(sc, use_bvh=True).render(PATCH_CAM, W, H, K, 0.0, 0.05)
    failures = 0
    n = 0
    while True:
        rcp.rcp_debug_set(rcp.RCP_DEBUG_FAIL_ALLOC_AFTER, n)
        try:
            s = rcp.Scene(sc)
        except rcp.RcpError as e:
            assert e.status == rcp.RCP_ERR_OUT_OF_MEMORY, str(e)
            failures += 1
            n += 1
            assert n < 200, "the build kept failing"
            continue
        finally:
            rcp.rcp_debug_set(rcp.RCP_DEBUG_FAIL_ALLOC_AFTER, -1)
        break
    say("scene build failed at", failures, "allocation points before succeeding")
    assert failures >= 5
    # the render's first workspace allocation fails, later ones succeed
    for engine in (rcp.RCP_ENGINE_CHAIN, rcp.RCP_ENGINE_PASSES):
        s.set_engine(engine)
        img = torch.empty((K, H, W, 3), device="cuda")
        ids = torch.empty((K, H, W), dtype=torch.int32, device="cuda")
        big_H = 64 * (engine + 2)
        rcp.rcp_debug_set(rcp.RCP_DEBUG_FAIL_ALLOC_AFTER, 0)
        try:
            with pytest.raises(rcp.RcpError) as e:
                rcp.rcp_render(s.handle, PATCH_CAM, W, big_H, K, rcp.make_displacement(0.0, 0.05), torch.empty(
                    (K, big_H, W, 3), device="cuda"), None)
            assert e.value.status == rcp.RCP_ERR_OUT_OF_MEMORY
        finally:
            rcp.rcp_debug_set(rcp.RCP_DEBUG_FAIL_ALLOC_AFTER, -1)
        rcp.rcp_render(s.handle, PATCH_CAM, W, H, K, rcp.make_displacement(0.0, 0.05), img, ids)
        torch.cuda.synchronize()
        assert np.array_equal(img.cpu().numpy(), o_img) and np.array_equal(ids.cpu().numpy(), o_ids), engine
    # a server whose slot buffers cannot be allocated is not created
    rcp.rcp_debug_set(rcp.RCP_DEBUG_FAIL_ALLOC_AFTER, 1)
    try:
        with pytest.raises(rcp.RcpError) as e:
            rcp.rcp_server_create(s.handle, 1 << 24, max_inflight=2)
        assert e.value.status == rcp.RCP_ERR_OUT_OF_MEMORY
    finally:
        rcp.rcp_debug_set(rcp.RCP_DEBUG_FAIL_ALLOC_AFTER, -1)
    srv = rcp.rcp_server_create(s.handle, 1 << 24, max_inflight=2)
    rcp.rcp_server_destroy(srv)
    s.close()
