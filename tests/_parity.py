"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np

# The stated bar: hit IDs bit-exact in the first rendered image; after the K
# passes a mean absolute RGB error <= 1e-3 and at most 0.1% of pixels with a
# channel off by more than 1/255.
MEAN_ABS_TOL = 1e-3
FRAC_OFF_TOL = 1e-3
OFF = 1.0 / 255.0


def parity_report(g_img, g_ids, o_img, o_ids):
    err = np.abs(g_img.astype(np.float64) - o_img.astype(np.float64))
    return {
        "ids0_equal": bool(np.array_equal(g_ids[0], o_ids[0])),
        "mean_abs": float(err.mean()) if err.size else 0.0,
        "frac_off_last": float(np.mean(np.any(err[-1] > OFF, axis=-1))) if err.size else 0.0,
        "exact_images": bool(np.array_equal(g_img, o_img)),
        "exact_ids": bool(np.array_equal(g_ids, o_ids)),
        "n_pix_diff": int(np.sum(np.any(g_img != o_img, axis=-1))),
    }


def assert_parity(g_img, g_ids, o_img, o_ids, label=""):
    r = parity_report(g_img, g_ids, o_img, o_ids)
    assert r["ids0_equal"], (label, r)
    assert r["mean_abs"] <= MEAN_ABS_TOL, (label, r)
    assert r["frac_off_last"] <= FRAC_OFF_TOL, (label, r)
    return r
