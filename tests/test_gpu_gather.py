"""GPU parity of the screen-space variant (Section 6, edges Section 6.1):
bit-exact against the oracle (the path copies colours; only the source
index is computed, in the same FP32 operations on both sides)."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_2312_12392_amd import rcp

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    rcp.load()


def run_gather(img, n, smudge, edge, centred):
    H, W = img.shape[:2]
    t_in = torch.from_numpy(np.ascontiguousarray(img, np.float32)).cuda()
    out = torch.empty((n, H, W, 3), device="cuda")
    rcp.rcp_gather_passes(t_in, W, H, n, smudge, edge, centred, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("edge", [rcp.RCP_EDGE_CLAMP, rcp.RCP_EDGE_WRAP, rcp.RCP_EDGE_MIRROR])
@pytest.mark.parametrize("W,H,n,smudge,centred,seed", [
    (64, 64, 6, 3.0, True, 0), (67, 45, 4, 7.5, True, 1), (1, 1, 3, 5.0, True, 2), (130, 1, 2, 40.0, True, 3),
    (1, 77, 2, 40.0, False, 4), (33, 21, 5, 0.0, True, 5), (50, 40, 3, 250.0, True, 6), (19, 23, 4, 2.0, False, 7),
])
def test_gather_matches_oracle(edge, W, H, n, smudge, centred, seed):
    say("gather", edge, W, H, n, smudge, centred)
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, size=(H, W, 3)).astype(np.float32)
    img.reshape(-1, 3)[::7, :2] = [0.0, 1.0]
    img.reshape(-1, 3)[1::5, :2] = 0.5
    g = run_gather(img, n, smudge, edge, centred)
    o = oracle.gather(img, n, smudge, edge=edge, centred=centred)
    assert np.array_equal(g, o)


@pytest.mark.parametrize("edge", [rcp.RCP_EDGE_CLAMP, rcp.RCP_EDGE_WRAP, rcp.RCP_EDGE_MIRROR])
def test_gather_on_a_rendered_frame(edge):
    """The variant's intended input: the first (undisplaced) render."""
    w = scenegen.workload("terrain1m")
    say("gather rendered", edge)
    W, H = 640, 360
    s = rcp.Scene(w.scene)
    imgs, _ = s.render(w.camera, W, H, 1, 0.0, 0.0)
    torch.cuda.synchronize()
    base = imgs[0].cpu().numpy()
    g = run_gather(base, 5, 6.0, edge, True)
    o = oracle.gather(base, 5, 6.0, edge=edge, centred=True)
    assert np.array_equal(g, o)
    s.close()
