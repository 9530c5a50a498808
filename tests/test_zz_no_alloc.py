"""rcp_render_noalloc (the entry point for callers that cannot allocate)
against rcp_render, through the C ABI: two calls in a row, the second on a
smaller input, each bit-exact against rcp_render of the same arguments (and,
on the small scene, against the oracle), in every displacement mode."""
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


def both(s, cam, W, H, K, d):
    a = torch.full((K, H, W, 3), -1.0, device="cuda")
    ai = torch.full((K, H, W), -7, dtype=torch.int32, device="cuda")
    rcp.rcp_render_noalloc(s.handle, cam, W, H, K, d, a, ai)
    b = torch.empty_like(a)
    bi = torch.empty_like(ai)
    rcp.rcp_render(s.handle, cam, W, H, K, d, b, bi)
    torch.cuda.synchronize()
    return a, ai, b, bi


def test_scratch_size_is_stated():
    assert rcp.rcp_render_noalloc_scratch_bytes() == 64 << 20


@pytest.mark.parametrize("mode,z0", [(rcp.RCP_MODE_COLOR, 0.0), (rcp.RCP_MODE_DEPTH, 1.2),
                                     (rcp.RCP_MODE_NORMAL, 0.0)])
def test_noalloc_equals_render_twice_second_smaller(mode, z0):
    sc = scenegen.terrain_patch(12, 40, 20)
    s = rcp.Scene(sc)
    orc = oracle.OracleScene(sc, use_bvh=True)
    d = rcp.make_displacement(0.01, 0.05, mode, z0)
    for (W, H, K) in [(203, 151, 6), (37, 29, 3)]:
        say("noalloc", mode, W, H, K)
        a, ai, b, bi = both(s, PATCH_CAM, W, H, K, d)
        assert torch.equal(a, b) and torch.equal(ai, bi), (W, H, K)
        o, oi = orc.render(PATCH_CAM, W, H, K, 0.01, 0.05, mode=mode, z0=z0)
        assert np.array_equal(a.cpu().numpy(), o) and np.array_equal(ai.cpu().numpy(), oi)
    s.close()


def test_noalloc_full_size_frame_twice():
    """The benchmark frame (1080p, K=6, 1M triangles), then a smaller one."""
    w = scenegen.workload("terrain1m")
    s = rcp.Scene(w.scene)
    d = rcp.make_displacement(w.lambda_eye, w.lambda_dir)
    for (W, H, K) in [(w.width, w.height, w.passes), (640, 360, 4)]:
        say("noalloc terrain1m", W, H, K)
        a, ai, b, bi = both(s, w.camera, W, H, K, d)
        assert torch.equal(a, b) and torch.equal(ai, bi), (W, H, K)
    rcp.rcp_check(s.handle)
    s.close()


def test_noalloc_rejects_invalid_arguments():
    w = scenegen.workload("soup256")
    s = rcp.Scene(w.scene)
    d = rcp.make_displacement(0.0, 0.02)
    out = torch.empty((2, 8, 8, 3), device="cuda")
    for K in (0, 65):
        with pytest.raises(rcp.RcpError) as e:
            rcp.rcp_render_noalloc(s.handle, w.camera, 8, 8, K, d, out)
        assert e.value.status == rcp.RCP_ERR_INVALID_ARGUMENT
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render_noalloc(s.handle, w.camera, 8, 8, 2, d, None)
    with pytest.raises(rcp.RcpError):
        rcp.rcp_render_noalloc(0, w.camera, 8, 8, 2, d, out)
    s.close()


def test_noalloc_beyond_the_order_area_then_within():
    """A view of more than 2^16 tiles (screen order: the scratch's order area
    holds 2^16), then a smaller one (cost order), each equal to rcp_render."""
    sc = scenegen.terrain_patch(12, 40, 20)
    s = rcp.Scene(sc)
    d = rcp.make_displacement(0.01, 0.05)
    for (W, H, K) in [(2600, 1800, 2), (1920, 1080, 2)]:
        say("noalloc order area", W, H, K)
        a, ai, b, bi = both(s, PATCH_CAM, W, H, K, d)
        assert torch.equal(a, b) and torch.equal(ai, bi), (W, H, K)
    s.close()
