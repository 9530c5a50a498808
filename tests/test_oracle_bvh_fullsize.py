"""The oracle's BVH against its brute-force definition on the full-size scenes.

Every full-size parity check of the HIP path compares against the oracle
with its BVH, so the BVH must give exactly the brute-force answer (Section 2:
the render is the closest surface each pixel's camera sees): the same hit
distance, triangle and side, bit for bit, or a miss on both.  The smaller
pins cover scenes of up to 1,500 triangles; here the 1M- and 4M-triangle
terrain scenes are queried with rays of every kind the renders produce, and
with rays built to graze the tree's box planes:

* pinhole rays of the benchmark camera;
* displaced rays (random previous colours; previous colours at the extremes
  0 and 1 with a large displacement of eye and direction);
* vertical rays through scene vertices (edge functions exactly zero);
* rays lying in the terrain's grid planes x = const and z = const, through a
  vertex (they run along box faces);
* rays from the eye aimed at scene vertices;
* nearly horizontal rays just above the terrain;
* rays tilted by 1e-10 .. 1e-4 out of the plane of a triangle they cross
  (ill-conditioned hit distances).
"""
import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.slow


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def ray_classes(w, n_each, seed):
    """Seeded rays of each kind: dict name -> (origins [n][3], directions [n][3]) float32."""
    rng = np.random.default_rng(seed)
    sc = w.scene
    W, H = w.width, w.height
    out = {}

    def camera_rays(prev_fn, le, ld):
        pix = rng.choice(W * H, size=n_each, replace=False)
        O = np.zeros((n_each, 3), np.float32)
        D = np.zeros((n_each, 3), np.float32)
        for i, p in enumerate(pix):
            y, x = divmod(int(p), W)
            O[i], D[i] = oracle.ray(w.camera, W, H, x, y, prev_fn(), le, ld)
        return O, D

    out["pinhole"] = camera_rays(lambda: [0.5, 0.5, 0.5], 0.0, 0.0)
    out["displaced_random"] = camera_rays(lambda: rng.uniform(0, 1, 3), 0.0, w.lambda_dir)
    out["displaced_extreme"] = camera_rays(lambda: rng.integers(0, 2, 3).astype(np.float32), 0.05, 0.5)

    V = sc.verts.astype(np.float32)
    tgt = V[rng.choice(V.shape[0], size=n_each, replace=False)]
    out["vertical_through_vertices"] = ((tgt + np.float32([0, 1, 0])).astype(np.float32),
                                        np.tile(np.float32([0, -1, 0]), (n_each, 1)))
    O = tgt.astype(np.float64)
    O[:, 1] += rng.uniform(0.05, 0.5, n_each)
    O[:, 2] += rng.uniform(-0.5, 0.5, n_each)
    D = tgt - O
    D[:, 0] = 0.0
    out["grid_plane_x"] = (O.astype(np.float32), _unit(D).astype(np.float32))
    O = tgt.astype(np.float64)
    O[:, 1] += rng.uniform(0.05, 0.5, n_each)
    O[:, 0] += rng.uniform(-0.5, 0.5, n_each)
    D = tgt - O
    D[:, 2] = 0.0
    out["grid_plane_z"] = (O.astype(np.float32), _unit(D).astype(np.float32))
    O = np.tile(np.asarray(w.camera.eye, np.float32), (n_each, 1))
    out["eye_to_vertex"] = (O, _unit(tgt.astype(np.float64) - O).astype(np.float32))
    O = tgt.astype(np.float64)
    O[:, 1] += rng.uniform(1e-4, 2e-3, n_each)
    ang = rng.uniform(0, 2 * np.pi, n_each)
    D = np.stack([np.cos(ang), -rng.uniform(0, 0.02, n_each), np.sin(ang)], -1)
    out["grazing"] = (O.astype(np.float32), _unit(D).astype(np.float32))

    # through a random point of a random triangle, tilted slightly out of its plane
    T = rng.choice(sc.idx.shape[0], size=n_each)
    tri = sc.verts.astype(np.float64)[sc.idx[T].astype(np.int64)]
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    nrm = _unit(np.cross(e1, e2))
    P = (rng.dirichlet([1, 1, 1], size=n_each)[:, :, None] * tri).sum(1)
    a = rng.normal(size=(n_each, 2))
    d = _unit(a[:, :1] * e1 + a[:, 1:] * e2)
    tilt = np.exp(rng.uniform(np.log(1e-10), np.log(1e-4), n_each)) * rng.choice([-1, 1], n_each)
    d = _unit(d + tilt[:, None] * nrm)
    o = P - rng.uniform(0.0005, 0.3, n_each)[:, None] * d
    out["in_plane"] = (o.astype(np.float32), d.astype(np.float32))
    return out


def _check_scene(name, n_each, seed):
    w = scenegen.workload(name)
    ob = oracle.OracleScene(w.scene, use_bvh=True)
    classes = ray_classes(w, n_each, seed)
    hits = 0
    for cls, (O, D) in classes.items():
        t_b, i_b, f_b = ob.closest_hits(O, D, brute=False)
        t_f, i_f, f_f = ob.closest_hits(O, D, brute=True)
        same = (np.array_equal(t_b.view(np.uint32), t_f.view(np.uint32)) and np.array_equal(i_b, i_f)
                and np.array_equal(f_b, f_f))
        bad = np.nonzero((t_b.view(np.uint32) != t_f.view(np.uint32)) | (i_b != i_f) | (f_b != f_f))[0]
        assert same, (name, cls, bad[:10], i_b[bad[:5]], i_f[bad[:5]])
        hits += int((i_f >= 0).sum())
    # the rays must actually meet the scene
    assert hits > 0.6 * n_each * len(classes), hits
    ob.close()


def test_bvh_equals_bruteforce_terrain1m(oracle_lib):
    _check_scene("terrain1m", 400, 0)


def test_bvh_equals_bruteforce_terrain4m(oracle_lib):
    _check_scene("terrain4m", 120, 1)
