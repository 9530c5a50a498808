"""Full-size workloads beyond the 1080p frame, in the configuration the
benchmark runs them: sampled pixels checked through their whole K-pass
chains against the oracle.

* the 16M-triangle scene, 3840x2160, K=8, on frames of the spline
  walk-through;
* the 4M-triangle scene behind the continuous-batching server: a burst of
  requests from the served trace (mixed resolution and pass count), each
  result checked on sampled pixels."""
import time

import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_2312_12392_amd import rcp

from _parity import assert_parity

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    rcp.load()


def sampled(orc, imgs, ids, cam, W, H, K, le, ld, pix, name):
    P = W * H
    pt = torch.from_numpy(pix.astype(np.int64)).cuda()
    g_img = imgs.reshape(K, P, 3)[:, pt].cpu().numpy()
    g_ids = ids.reshape(K, P)[:, pt].cpu().numpy()
    o_img, o_ids = orc.render_pixels(cam, W, H, K, le, ld, pix.astype(np.int32))
    r = assert_parity(g_img, g_ids, o_img.transpose(1, 0, 2), o_ids.T, name)
    assert r["exact_images"] and r["exact_ids"], r


def test_terrain16m_walkthrough_frames_sampled():
    w = scenegen.workload("terrain16m")
    say("terrain16m", w.scene.n_tris, w.width, w.height, w.passes)
    s = rcp.Scene(w.scene)
    orc = oracle.OracleScene(w.scene, use_bvh=True)
    W, H, K = w.width, w.height, w.passes
    pts = scenegen.spline_path(7)
    rng = np.random.default_rng(16)
    for frame in (0, 37, 119):
        cam = scenegen.walk_camera(pts, frame / 120)
        say("frame", frame)
        imgs, ids = s.render(cam, W, H, K, 0.0, w.lambda_dir)
        torch.cuda.synchronize()
        pix = np.unique(np.concatenate([rng.choice(W * H, size=3000, replace=False),
                                        np.arange(W) + W * (H // 2)]))          # plus one full row
        sampled(orc, imgs, ids, cam, W, H, K, 0.0, w.lambda_dir, pix, f"terrain16m frame {frame}")
    s.close()


def test_served_terrain4m_burst_sampled():
    w = scenegen.workload("terrain4m")
    say("terrain4m served", w.scene.n_tris)
    s = rcp.Scene(w.scene)
    orc = oracle.OracleScene(w.scene, use_bvh=True)
    trace = scenegen.served_trace(5, 200.0, 0.1)[:10]
    srv = rcp.rcp_server_create(s.handle, 8 << 30, max_inflight=2)
    d = rcp.make_displacement(0.0, w.lambda_dir)
    tickets = [rcp.rcp_submit(srv, cam, W, H, K, d, with_ids=True) for (_, cam, W, H, K) in trace]
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            st, _ = rcp.rcp_poll(srv, t)
            assert st != rcp.RCP_REQ_FAILED
            if st == rcp.RCP_REQ_DONE:
                pending.discard(t)
        assert time.time() - t0 < 60, "requests did not finish"
        time.sleep(0.001)
    rng = np.random.default_rng(4)
    for (_, cam, W, H, K), t in zip(trace, tickets):
        say("request", W, H, K)
        img = torch.empty((K, H, W, 3), device="cuda")
        ids = torch.empty((K, H, W), dtype=torch.int32, device="cuda")
        rcp.rcp_result_copy(srv, t, img, ids)
        torch.cuda.synchronize()
        pix = rng.choice(W * H, size=min(W * H, 800), replace=False)
        sampled(orc, img, ids, cam, W, H, K, 0.0, w.lambda_dir, pix, f"served {W}x{H} K={K}")
        rcp.rcp_release(srv, t)
    rcp.rcp_server_destroy(srv)
    s.close()
