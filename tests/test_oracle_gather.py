"""Pins for the oracle's screen-space variant (Section 6) and its edge rules
(Section 6.1), against numpy's roll and pad and hand-computed cases."""
import numpy as np
import pytest

import oracle

CLAMP, WRAP, MIRROR = oracle.EDGE_CLAMP, oracle.EDGE_WRAP, oracle.EDGE_MIRROR
NP_PAD = {CLAMP: "edge", WRAP: "wrap", MIRROR: "symmetric"}


def shifted(img, dx, dy, edge):
    """Image whose pixel (x, y) is img at (x + dx, y + dy), numpy edge rule."""
    H, W = img.shape[:2]
    m = max(abs(dx), abs(dy)) + 1
    p = np.pad(img, ((m, m), (m, m), (0, 0)), mode=NP_PAD[edge])
    return p[m + dy:m + dy + H, m + dx:m + dx + W]


@pytest.mark.parametrize("edge", [CLAMP, WRAP, MIRROR])
@pytest.mark.parametrize("r,g,smudge", [(1.0, 0.5, 3.0), (0.0, 0.5, 2.0), (0.5, 1.0, 4.0), (0.5, 0.0, 1.0),
                                        (1.0, 1.0, 2.0), (0.75, 0.25, 4.0)])
def test_uniform_red_green_is_a_shift(oracle_lib, edge, r, g, smudge):
    """Pixels sharing R and G all move by the same offset (blue does not move
    anything here), so one pass is a shift of the image: right for R = 1,
    up (towards row 0) for G = 1."""
    rng = np.random.default_rng(0)
    H, W = 13, 17
    img = np.empty((H, W, 3), np.float32)
    img[..., 0] = r
    img[..., 1] = g
    img[..., 2] = rng.uniform(0, 1, size=(H, W))
    out = oracle.gather(img, 1, smudge, edge=edge)[0]
    dx = int(np.floor(0.5 + (2 * r - 1) * smudge))
    dy = int(np.floor(0.5 - (2 * g - 1) * smudge))
    assert np.array_equal(out, shifted(img, dx, dy, edge))


def test_literal_red_green_offsets(oracle_lib):
    rng = np.random.default_rng(1)
    H, W = 9, 11
    img = np.empty((H, W, 3), np.float32)
    img[..., 0] = 1.0
    img[..., 1] = 0.0
    img[..., 2] = rng.uniform(0, 1, size=(H, W))
    out = oracle.gather(img, 1, 2.0, edge=WRAP, centred=False)[0]
    assert np.array_equal(out, shifted(img, 2, 0, WRAP))


def test_neutral_and_zero_smudge_do_not_move(oracle_lib):
    rng = np.random.default_rng(2)
    img = rng.uniform(0, 1, size=(10, 12, 3)).astype(np.float32)
    for edge in (CLAMP, WRAP, MIRROR):
        assert np.array_equal(oracle.gather(img, 3, 0.0, edge=edge)[-1], img)
        grey = img.copy()
        grey[..., :2] = 0.5
        assert np.array_equal(oracle.gather(grey, 2, 5.0, edge=edge)[-1], grey)


def test_edge_rules_by_hand(oracle_lib):
    """One row; the left-most pixel asks for the pixel two to its left."""
    W = 5
    img = np.zeros((1, W, 3), np.float32)
    img[0, :, 2] = np.arange(W)            # blue marks the source column
    img[0, :, 1] = 0.5
    img[0, 0, 0] = 0.0                      # centred red -1: two pixels left with smudge 2
    out = {e: oracle.gather(img, 1, 2.0, edge=e)[0, 0, 0, 2] for e in (CLAMP, WRAP, MIRROR)}
    assert out[CLAMP] == 0.0                # clamped to column 0
    assert out[WRAP] == 3.0                 # -2 wraps to W - 2
    assert out[MIRROR] == 1.0               # -2 mirrors to 1 (-1 -> 0, -2 -> 1)


def test_passes_chain(oracle_lib):
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, size=(16, 20, 3)).astype(np.float32)
    out = oracle.gather(img, 4, 3.0)
    for k in range(1, 4):
        assert np.array_equal(out[k], oracle.gather(out[k - 1], 1, 3.0)[0])
    # every output colour is one of the input's colours
    cols = {tuple(c) for c in img.reshape(-1, 3)}
    assert all(tuple(c) in cols for c in out[-1].reshape(-1, 3))
