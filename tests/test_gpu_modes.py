"""GPU parity of the depth (Section 4) and normal (Section 5) mappings.

Same bar as the colour mapping (pass-1 hit IDs bit-exact; mean |dRGB| <=
1e-3 and <= 0.1% of pixels off by more than 1/255 after K passes), and the
path is again expected to match the oracle bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from _parity import assert_parity
from paper_2312_12392_amd import rcp

pytestmark = pytest.mark.gpu

DEPTH, NORMAL = rcp.RCP_MODE_DEPTH, rcp.RCP_MODE_NORMAL
AXIS_CAM = scenegen.camera_look_at([0, 0, -3], [0, 0, 0], [0, 1, 0], 60.0)
PATCH_CAM = scenegen.camera_look_at([0, 0.5, -1.4], [0, 0.05, 0], [0, 1, 0], 60.0)
OBLIQUE_CAM = scenegen.camera_look_at([1.3, -0.7, 1.9], [0.05, 0.1, -0.1], [0.2, 1, 0.1], 75.0)


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    rcp.load()


@pytest.mark.parametrize("mode", [DEPTH, NORMAL])
@pytest.mark.parametrize("cam,W,H,le,ld,z0,seed", [
    (PATCH_CAM, 67, 45, 0.01, 0.05, 1.2, 1),
    (OBLIQUE_CAM, 31, 17, 0.3, 0.9, 2.5, 2),
    (AXIS_CAM, 1920, 1080, 0.0, 0.01, 3.0, 4),
])
def test_generate_rays_bit_exact_modes(mode, cam, W, H, le, ld, z0, seed):
    say("generate_rays mode", mode, W, H)
    rng = np.random.default_rng(seed)
    prev = rng.uniform(0, 1, size=(H, W, 3)).astype(np.float32)
    aux = np.empty((H, W, 4), np.float32)
    aux[..., 0] = rng.uniform(0.2, 5.0, size=(H, W))
    n = rng.normal(size=(H, W, 3))
    aux[..., 1:] = n / np.linalg.norm(n, axis=-1, keepdims=True)
    flat = aux.reshape(-1, 4)
    flat[::6] = [np.inf, 0, 0, 0]            # misses
    flat[1::9, 0] = np.float32(z0)           # in focus
    org = torch.empty((H, W, 3), device="cuda")
    dirs = torch.empty((H, W, 3), device="cuda")
    rcp.rcp_generate_rays(cam, W, H, rcp.make_displacement(le, ld, mode, z0), torch.from_numpy(prev).cuda(), org,
                          dirs, prev_aux=torch.from_numpy(aux).cuda())
    torch.cuda.synchronize()
    g_o = org.cpu().numpy().reshape(-1, 3)
    g_d = dirs.cpu().numpy().reshape(-1, 3)
    P = W * H
    pix = np.arange(P) if P <= 5000 else rng.choice(P, size=4000, replace=False)
    for p in pix:
        y, x = divmod(int(p), W)
        o, d = oracle.ray(cam, W, H, x, y, prev[y, x], le, ld, prev_aux=aux[y, x], mode=mode, z0=z0)
        assert np.array_equal(g_o[p], o) and np.array_equal(g_d[p], d), (x, y)


RENDER_CASES = [
    ("soup256", lambda: scenegen.soup_scene(0, 256), AXIS_CAM, 64, 64, 6, 0.0, 0.02, 3.0),
    ("patch_ragged", lambda: scenegen.terrain_patch(11, 24, 8), PATCH_CAM, 67, 45, 5, 0.0, 0.05, 1.2),
    ("patch_eye", lambda: scenegen.terrain_patch(12, 40, 20), PATCH_CAM, 96, 72, 6, 0.03, 0.2, 1.0),
    ("oblique_soup", lambda: scenegen.soup_scene(9, 1500), OBLIQUE_CAM, 80, 48, 6, 0.01, 0.05, 2.4),
    ("adversarial", lambda: scenegen.adversarial_scene(), AXIS_CAM, 50, 41, 6, 0.0, 0.1, 3.2),
    ("empty", lambda: scenegen.empty_scene(), AXIS_CAM, 23, 19, 3, 0.0, 0.1, 1.0),
]


@pytest.mark.parametrize("engine", [rcp.RCP_ENGINE_CHAIN, rcp.RCP_ENGINE_PASSES], ids=["chain", "passes"])
@pytest.mark.parametrize("mode", [DEPTH, NORMAL])
@pytest.mark.parametrize("case", RENDER_CASES, ids=[c[0] for c in RENDER_CASES])
def test_render_modes_match_oracle(mode, case, engine):
    name, scene_fn, cam, W, H, K, le, ld, z0 = case
    say("render mode", mode, name, "engine", engine)
    sc = scene_fn()
    s = rcp.Scene(sc)
    s.set_engine(engine)
    imgs, ids = s.render(cam, W, H, K, le, ld, mode=mode, z0=z0)
    torch.cuda.synchronize()
    g_img, g_ids = imgs.cpu().numpy(), ids.cpu().numpy()
    s.close()
    o_img, o_ids = oracle.OracleScene(sc, use_bvh=True).render(cam, W, H, K, le, ld, mode=mode, z0=z0)
    r = assert_parity(g_img, g_ids, o_img, o_ids, name)
    assert r["exact_images"] and r["exact_ids"], r


@pytest.mark.parametrize("mode", [DEPTH, NORMAL, rcp.RCP_MODE_COLOR])
def test_render_pass_chain_with_hit_data(mode):
    say("render_pass chain mode", mode)
    sc = scenegen.terrain_patch(11, 24, 8)
    W, H, K, z0 = 61, 47, 5, 1.2
    s = rcp.Scene(sc)
    imgs, ids = s.render(PATCH_CAM, W, H, K, 0.01, 0.05, mode=mode, z0=z0)
    d = rcp.make_displacement(0.01, 0.05, mode, z0)
    o = oracle.OracleScene(sc, use_bvh=True)
    prev, prev_aux = None, None
    o_prev, o_aux = None, None
    for k in range(K):
        out = torch.empty((H, W, 3), device="cuda")
        oid = torch.empty((H, W), dtype=torch.int32, device="cuda")
        aux = torch.empty((H, W, 4), device="cuda")
        rcp.rcp_render_pass(s.handle, PATCH_CAM, W, H, d, prev, out, oid, prev_aux=prev_aux, out_aux=aux)
        torch.cuda.synchronize()
        assert torch.equal(out, imgs[k]) and torch.equal(oid, ids[k]), k
        r_img, r_ids, r_aux = o.render_pass(PATCH_CAM, W, H, 0.01, 0.05, prev=o_prev, prev_aux=o_aux, mode=mode,
                                            z0=z0, with_aux=True)
        assert np.array_equal(aux.cpu().numpy(), r_aux), k
        prev, prev_aux = out, aux
        o_prev, o_aux = r_img, r_aux
    s.close()
