"""Seeded synthetic inputs for the recursive camera-painting renderer.

This module produces scenes (triangle soups, fBm terrain with boxes), base
cameras and the small analytic scenes used by the tests.  It holds none of
the method's arithmetic: no ray generation, no displacement, no intersection
and no shading.  Both the CPU oracle and the HIP library consume its output,
and nothing else is shared between them.

All random draws use ``numpy.random.default_rng(seed)`` (PCG64) in the order
written in each generator.  Every array is returned as float32 / uint32, so
both consumers read identical bits.

The paper publishes no scenes (its OptiX examples used a textured
environment sphere, Section 6), so the workloads here are synthetic
stand-ins with the shapes, sizes and structure of the stated configurations:
a 256-triangle random soup, and fBm terrains of about 1M / 4M / 16M
triangles with randomly placed, scaled and rotated boxes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "Camera", "Workload", "camera_look_at", "soup_scene",
    "terrain_scene", "workload", "quad_scene", "halfplane_scene",
    "random_soup", "terrain_patch", "adversarial_scene", "empty_scene",
    "DEFAULT_LIGHT", "DEFAULT_BACKGROUND",
]


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.sqrt(np.dot(v, v))


# Directional light (pointing toward the light) and miss colour.  The paper
# leaves both unspecified; the background is the neutral grey so that a
# missed ray is not displaced on the following pass (Section 3).
DEFAULT_LIGHT = _unit([0.3, 0.8, -0.5]).astype(np.float32)
DEFAULT_BACKGROUND = np.array([0.5, 0.5, 0.5], dtype=np.float32)


@dataclass
class Scene:
    """Triangle scene: shared vertices, index triples, per-triangle albedo."""
    verts: np.ndarray               # float32 [Nv, 3]
    idx: np.ndarray                 # uint32  [Nt, 3]
    rgb: np.ndarray                 # float32 [Nt, 3], albedo in [0, 1]
    light: np.ndarray = field(default_factory=lambda: DEFAULT_LIGHT.copy())
    k_a: float = 0.0
    k_d: float = 1.0
    background: np.ndarray = field(default_factory=lambda: DEFAULT_BACKGROUND.copy())
    name: str = "scene"

    def __post_init__(self):
        self.verts = np.ascontiguousarray(self.verts, dtype=np.float32).reshape(-1, 3)
        self.idx = np.ascontiguousarray(self.idx, dtype=np.uint32).reshape(-1, 3)
        self.rgb = np.ascontiguousarray(self.rgb, dtype=np.float32).reshape(-1, 3)
        self.light = np.ascontiguousarray(self.light, dtype=np.float32).reshape(3)
        self.background = np.ascontiguousarray(self.background, dtype=np.float32).reshape(3)
        assert self.idx.shape[0] == self.rgb.shape[0]

    @property
    def n_tris(self) -> int:
        return int(self.idx.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])


@dataclass
class Camera:
    """Base pinhole camera: eye, orthonormal basis and tan(vfov / 2)."""
    eye: np.ndarray
    right: np.ndarray
    up: np.ndarray
    forward: np.ndarray
    tan_half_fovy: float

    def __post_init__(self):
        for k in ("eye", "right", "up", "forward"):
            setattr(self, k, np.ascontiguousarray(getattr(self, k), dtype=np.float32).reshape(3))
        self.tan_half_fovy = float(np.float32(self.tan_half_fovy))


@dataclass
class Workload:
    """A render job: scene, base camera, image size, pass count, lambdas."""
    scene: Scene
    camera: Camera
    width: int
    height: int
    passes: int
    lambda_eye: float
    lambda_dir: float
    name: str = "workload"

    @property
    def nominal_rays(self) -> int:
        return self.width * self.height * self.passes


def camera_look_at(eye, target, up, vfov_deg) -> Camera:
    """Camera basis computed in double and rounded once to float32.

    forward = normalize(target - eye); right = normalize(up x forward);
    up' = forward x right.  For an eye looking along +z with up +y this gives
    right = +x, up = +y.
    """
    eye = np.asarray(eye, dtype=np.float64)
    f = _unit(np.asarray(target, dtype=np.float64) - eye)
    r = _unit(np.cross(np.asarray(up, dtype=np.float64), f))
    u = np.cross(f, r)
    u = _unit(u)
    th = math.tan(math.radians(vfov_deg) * 0.5)
    return Camera(eye=eye, right=r, up=u, forward=f, tan_half_fovy=th)


# --------------------------------------------------------------------------
# Random triangle soup (the 256-triangle correctness scene)
# --------------------------------------------------------------------------

def soup_scene(seed: int = 0, n: int = 256, extent: float = 0.5) -> Scene:
    """``n`` triangles with vertices uniform in [-extent, extent]^3.

    Draw order: vertices (n, 3, 3), then albedo (n, 3).
    """
    rng = np.random.default_rng(seed)
    v = rng.uniform(-extent, extent, size=(n, 3, 3))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    return Scene(verts=v.reshape(-1, 3), idx=np.arange(3 * n, dtype=np.uint32).reshape(n, 3),
                 rgb=rgb, name=f"soup{n}_s{seed}")


random_soup = soup_scene


# --------------------------------------------------------------------------
# fBm terrain + boxes
# --------------------------------------------------------------------------

def _gradient_noise_2d(x, y, perm):
    """2-D gradient noise with a quintic fade and 8 lattice gradient directions.

    ``perm`` is a permutation of 0..255 (drawn by the caller).  Returns values
    roughly in [-1, 1].
    """
    p = np.concatenate([perm, perm]).astype(np.int64)
    xi = np.floor(x).astype(np.int64)
    yi = np.floor(y).astype(np.int64)
    xf = x - xi
    yf = y - yi
    xi &= 255
    yi &= 255
    ang = np.arange(8) * (np.pi / 4.0)
    gx = np.cos(ang)
    gy = np.sin(ang)

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def grad(h, dx, dy):
        h = h & 7
        return gx[h] * dx + gy[h] * dy

    aa = p[p[xi] + yi]
    ab = p[p[xi] + yi + 1]
    ba = p[p[xi + 1] + yi]
    bb = p[p[xi + 1] + yi + 1]
    u = fade(xf)
    v = fade(yf)
    n00 = grad(aa, xf, yf)
    n10 = grad(ba, xf - 1.0, yf)
    n01 = grad(ab, xf, yf - 1.0)
    n11 = grad(bb, xf - 1.0, yf - 1.0)
    nx0 = n00 + u * (n10 - n00)
    nx1 = n01 + u * (n11 - n01)
    return (nx0 + v * (nx1 - nx0)) * math.sqrt(2.0)


def _fbm(x, z, perm, octaves, base_cycles=4.0, lacunarity=2.0, gain=0.5):
    """fBm over the extent [-1, 1]: ``base_cycles`` lattice periods across it."""
    f = base_cycles / 2.0
    a = 1.0
    h = np.zeros(np.broadcast(x, z).shape, dtype=np.float64)
    for _ in range(octaves):
        h += a * _gradient_noise_2d((x + 1.0) * f, (z + 1.0) * f, perm)
        f *= lacunarity
        a *= gain
    return h


def _quat_to_mat(q):
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    m = np.empty(q.shape[:-1] + (3, 3))
    m[..., 0, 0] = 1 - 2 * (y * y + z * z)
    m[..., 0, 1] = 2 * (x * y - z * w)
    m[..., 0, 2] = 2 * (x * z + y * w)
    m[..., 1, 0] = 2 * (x * y + z * w)
    m[..., 1, 1] = 1 - 2 * (x * x + z * z)
    m[..., 1, 2] = 2 * (y * z - x * w)
    m[..., 2, 0] = 2 * (x * z - y * w)
    m[..., 2, 1] = 2 * (y * z + x * w)
    m[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return m


# Unit-cube corners and 12 outward-facing triangles (cross(v1-v0, v2-v0)
# points out of the box).
_CUBE_CORNERS = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], dtype=np.float64)
_CUBE_TRIS = np.array([
    [0, 1, 3], [0, 3, 2],      # x = -1
    [4, 6, 7], [4, 7, 5],      # x = +1
    [0, 4, 5], [0, 5, 1],      # y = -1
    [2, 3, 7], [2, 7, 6],      # y = +1
    [0, 2, 6], [0, 6, 4],      # z = -1
    [1, 5, 7], [1, 7, 3],      # z = +1
], dtype=np.int64)


def terrain_grid_cells(n_tris_target: int, n_boxes: int) -> int:
    """Cells per side so that 2 n^2 + 12 B is closest to the target count."""
    return int(round(math.sqrt((n_tris_target - 12 * n_boxes) / 2.0)))


def terrain_scene(seed: int, nominal_grid: int, n_tris_target: int, n_boxes: int,
                  height: float = 0.15, palette_size: int = 16, cells: int | None = None) -> Scene:
    """fBm heightfield on x, z in [-1, 1] plus randomly placed rotated boxes.

    Draw order from ``default_rng(seed)``: noise permutation (256), box
    centres (B, 2) in U[-0.95, 0.95], box half-extents (B, 3) in
    U[0.004, 0.02], box rotations (B, 4) standard normal (normalised
    quaternions), palette (P, 3) in U[0, 1], per-triangle palette index
    U{0..P-1} (Nt).

    The terrain has ``cells`` x ``cells`` quads (two triangles each); by
    default ``cells`` is chosen so that the total triangle count is closest
    to ``n_tris_target``.  ``nominal_grid`` N sets the octave count
    log2(N / 16) + 1, so the finest octave has a period of 4 nominal cells.
    Heights are min-max scaled to [0, ``height``].  Each box rests on the
    terrain: its centre sits one local y half-extent above the terrain
    height at its (x, z).
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(256)
    centres = rng.uniform(-0.95, 0.95, size=(n_boxes, 2))
    half = rng.uniform(0.004, 0.02, size=(n_boxes, 3))
    quat = rng.standard_normal(size=(n_boxes, 4))
    palette = rng.uniform(0.0, 1.0, size=(palette_size, 3))

    n = terrain_grid_cells(n_tris_target, n_boxes) if cells is None else int(cells)
    octaves = int(round(math.log2(nominal_grid / 16.0))) + 1
    g = np.linspace(-1.0, 1.0, n + 1)
    X, Z = np.meshgrid(g, g, indexing="ij")          # X[i, j] = g[i], Z[i, j] = g[j]
    H = _fbm(X, Z, perm, octaves)
    hmin, hmax = float(H.min()), float(H.max())
    scale = height / (hmax - hmin)
    H = (H - hmin) * scale
    verts_t = np.stack([X, H, Z], axis=-1).reshape(-1, 3)

    # Two triangles per cell, both with +y facing geometric normals.
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    v00 = (i * (n + 1) + j)
    v10 = ((i + 1) * (n + 1) + j)
    v01 = (i * (n + 1) + j + 1)
    v11 = ((i + 1) * (n + 1) + j + 1)
    t_a = np.stack([v00, v01, v10], axis=-1).reshape(-1, 3)
    t_b = np.stack([v10, v01, v11], axis=-1).reshape(-1, 3)
    tris_t = np.stack([t_a, t_b], axis=1).reshape(-1, 3)

    # Boxes.
    if n_boxes > 0:
        hc = (_fbm(centres[:, 0], centres[:, 1], perm, octaves) - hmin) * scale
        rot = _quat_to_mat(quat)                                   # (B, 3, 3)
        local = _CUBE_CORNERS[None, :, :] * half[:, None, :]       # (B, 8, 3)
        world = np.einsum("bij,bkj->bki", rot, local)
        ctr = np.stack([centres[:, 0], hc + half[:, 1], centres[:, 1]], axis=-1)
        world = world + ctr[:, None, :]
        verts_b = world.reshape(-1, 3)
        base = verts_t.shape[0] + np.arange(n_boxes)[:, None, None] * 8
        tris_b = (base + _CUBE_TRIS[None, :, :]).reshape(-1, 3)
        verts = np.concatenate([verts_t, verts_b], axis=0)
        tris = np.concatenate([tris_t, tris_b], axis=0)
    else:
        verts, tris = verts_t, tris_t

    pal_idx = rng.integers(0, palette_size, size=tris.shape[0])
    rgb = palette[pal_idx]
    return Scene(verts=verts, idx=tris.astype(np.uint32), rgb=rgb,
                 name=f"terrain{n}c_{n_boxes}b_s{seed}")


def terrain_patch(seed: int = 11, cells: int = 24, n_boxes: int = 8) -> Scene:
    """Small terrain (shared edges everywhere) for parity and watertightness."""
    return terrain_scene(seed, nominal_grid=64, n_tris_target=0, n_boxes=n_boxes, cells=cells)


# --------------------------------------------------------------------------
# Analytic and adversarial scenes for the tests
# --------------------------------------------------------------------------

def quad_scene(z0: float = 0.0, half: float = 1.0, rgb=(0.8, 0.6, 0.4)) -> Scene:
    """One square z = z0, |x|, |y| <= half, as two triangles facing -z."""
    v = np.array([[-half, -half, z0], [half, -half, z0], [half, half, z0], [-half, half, z0]])
    # cross(v1-v0, v2-v0) = (2h,0,0) x (2h,2h,0) = (0,0,4h^2): +z; reverse for -z.
    idx = np.array([[0, 2, 1], [0, 3, 2]])
    return Scene(verts=v, idx=idx, rgb=np.array([rgb, rgb]), name="quad")


def halfplane_scene(half: float = 4.0, left_rgb=(0.9, 0.1, 0.2), right_rgb=(0.2, 0.8, 0.3),
                    split_x: float = 0.0) -> Scene:
    """Plane z = 0 split at x = split_x into two differently coloured rectangles."""
    s = split_x
    v = np.array([[-half, -half, 0], [s, -half, 0], [s, half, 0], [-half, half, 0],
                  [s, -half, 0], [half, -half, 0], [half, half, 0], [s, half, 0]], dtype=np.float64)
    idx = np.array([[0, 2, 1], [0, 3, 2], [4, 6, 5], [4, 7, 6]])
    rgb = np.array([left_rgb, left_rgb, right_rgb, right_rgb])
    return Scene(verts=v, idx=idx, rgb=rgb, name="halfplane")


def adversarial_scene(seed: int = 5) -> Scene:
    """Axis-aligned flat triangles, shared edges, duplicates and degenerates.

    Includes: a fan of triangles sharing one vertex on the view axis, axis-
    aligned triangles in each coordinate plane, an exact duplicate triangle
    (tie in t, broken by the lower index), zero-area triangles (collinear and
    repeated vertices) and a grid of coplanar triangles sharing edges.
    """
    rng = np.random.default_rng(seed)
    vs = []
    ts = []

    def add(tri):
        base = sum(len(x) for x in vs)
        vs.append(np.asarray(tri, dtype=np.float64))
        ts.append([base, base + 1, base + 2])

    # Fan around the origin in the plane z = 0.3.
    m = 12
    for k in range(m):
        a0 = 2 * math.pi * k / m
        a1 = 2 * math.pi * (k + 1) / m
        add([[0, 0, 0.3], [0.4 * math.cos(a0), 0.4 * math.sin(a0), 0.3],
             [0.4 * math.cos(a1), 0.4 * math.sin(a1), 0.3]])
    # Axis-aligned triangles in the three coordinate planes.
    add([[-0.5, -0.5, 0.6], [-0.1, -0.5, 0.6], [-0.5, -0.1, 0.6]])
    add([[0.2, -0.6, 0.2], [0.2, -0.2, 0.2], [0.2, -0.6, 0.8]])      # plane x = 0.2
    add([[-0.6, 0.25, 0.1], [-0.2, 0.25, 0.1], [-0.6, 0.25, 0.7]])   # plane y = 0.25
    # Exact duplicate of the first fan triangle (same t everywhere).
    add(vs[0].copy())
    # Degenerate triangles: collinear and repeated vertices.
    add([[0.1, 0.1, 0.5], [0.2, 0.2, 0.5], [0.3, 0.3, 0.5]])
    add([[0.1, -0.1, 0.5], [0.1, -0.1, 0.5], [0.3, 0.2, 0.5]])
    add([[0.0, 0.0, 0.9], [0.0, 0.0, 0.9], [0.0, 0.0, 0.9]])
    # Coplanar grid with shared edges at z = 1.0 (behind the fan).
    g = 6
    xs = np.linspace(-0.7, 0.7, g + 1)
    for i in range(g):
        for j in range(g):
            p00 = [xs[i], xs[j], 1.0]
            p10 = [xs[i + 1], xs[j], 1.0]
            p01 = [xs[i], xs[j + 1], 1.0]
            p11 = [xs[i + 1], xs[j + 1], 1.0]
            add([p00, p10, p11])
            add([p00, p11, p01])
    verts = np.concatenate(vs, axis=0)
    idx = np.array(ts)
    rgb = rng.uniform(0.0, 1.0, size=(idx.shape[0], 3))
    return Scene(verts=verts, idx=idx, rgb=rgb, name="adversarial")


def empty_scene() -> Scene:
    return Scene(verts=np.zeros((0, 3)), idx=np.zeros((0, 3)), rgb=np.zeros((0, 3)), name="empty")


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

_SCENE_CACHE: dict = {}


def workload(name: str, literal_eye: bool = False) -> Workload:
    """Named workloads.

    ``soup256``      64x64, K=6, 256 random triangles, lambda = 0.02.
    ``terrain1m``    1920x1080, K=6, 1,000,418 triangles, lambda = 0.01.
    ``terrain4m``    the 4,001,672-triangle terrain (2048 nominal grid).
    ``terrain16m``   3840x2160, K=8, 15,995,442 triangles, lambda = 0.01.

    The colour mapping of Section 3 keeps the eye fixed, so lambda_eye = 0
    and lambda_dir = lambda.  ``literal_eye=True`` also displaces the eye by
    the same amount.
    """
    if name == "soup256":
        sc = _SCENE_CACHE.get(name) or soup_scene(0, 256)
        cam = camera_look_at([0, 0, -3], [0, 0, 0], [0, 1, 0], 60.0)
        lam = 0.02
        w, h, k = 64, 64, 6
    elif name == "terrain1m":
        sc = _SCENE_CACHE.get(name) or terrain_scene(1, 512, 1_000_000, 1000)
        cam = camera_look_at([0, 0.45, -1.25], [0, 0.05, 0], [0, 1, 0], 60.0)
        lam = 0.01
        w, h, k = 1920, 1080, 6
    elif name == "terrain4m":
        sc = _SCENE_CACHE.get(name) or terrain_scene(4, 2048, 4_000_000, 4000)
        cam = camera_look_at([0, 0.45, -1.25], [0, 0.05, 0], [0, 1, 0], 60.0)
        lam = 0.01
        w, h, k = 1920, 1080, 6
    elif name == "terrain16m":
        sc = _SCENE_CACHE.get(name) or terrain_scene(6, 4096, 16_000_000, 16000)
        cam = camera_look_at([0, 0.45, -1.25], [0, 0.05, 0], [0, 1, 0], 60.0)
        lam = 0.01
        w, h, k = 3840, 2160, 8
    else:
        raise KeyError(name)
    _SCENE_CACHE[name] = sc
    return Workload(scene=sc, camera=cam, width=w, height=h, passes=k,
                    lambda_eye=lam if literal_eye else 0.0, lambda_dir=lam, name=name)


# --------------------------------------------------------------------------
# View mixes for batched rendering
# --------------------------------------------------------------------------

BATCH_RESOLUTIONS = [(256, 256), (512, 512), (1280, 720), (1024, 1024)]


def orbit_views(seed: int = 3, n: int = 64, resolutions=None, k_range=(1, 8), target=(0.0, 0.0, 0.0)):
    """n views on a random orbit around the terrain: azimuth U[0, 2 pi),
    radius U[1.2, 1.6], height U[0.3, 0.6], looking at the origin, vfov 60;
    resolution uniform over ``resolutions``, K uniform in ``k_range``.

    Draw order from ``default_rng(seed)``: azimuth, radius, height (n each),
    resolution index (n), K (n).  Returns a list of (Camera, W, H, K)."""
    rng = np.random.default_rng(seed)
    res = list(resolutions or BATCH_RESOLUTIONS)
    az = rng.uniform(0.0, 2.0 * math.pi, size=n)
    rad = rng.uniform(1.2, 1.6, size=n)
    hgt = rng.uniform(0.3, 0.6, size=n)
    ri = rng.integers(0, len(res), size=n)
    ks = rng.integers(k_range[0], k_range[1] + 1, size=n)
    out = []
    for i in range(n):
        eye = [rad[i] * math.sin(az[i]), hgt[i], -rad[i] * math.cos(az[i])]
        cam = camera_look_at(eye, target, [0, 1, 0], 60.0)
        W, H = res[int(ri[i])]
        out.append((cam, int(W), int(H), int(ks[i])))
    return out


def _catmull_rom(P, u):
    """Point at parameter u in [0, len(P) - 3] of the centripetal-free
    (uniform) Catmull-Rom spline through control points P."""
    i = int(min(max(math.floor(u), 0), len(P) - 4))
    t = u - i
    p0, p1, p2, p3 = (np.asarray(P[i + k], dtype=np.float64) for k in range(4))
    return 0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t * t +
                  (-p0 + 3 * p1 - 3 * p2 + p3) * t * t * t)


def spline_path(seed: int, n_points: int = 16, height=(0.35, 0.65), extent: float = 0.8):
    """Control points of a walk-through: (x, z) uniform in [-extent, extent]^2,
    y in ``height`` (0.2-0.5 above the terrain's 0.15 maximum).  Draw order:
    x, z, y (n_points each)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-extent, extent, size=n_points)
    z = rng.uniform(-extent, extent, size=n_points)
    y = rng.uniform(height[0], height[1], size=n_points)
    return [np.array([x[i], y[i], z[i]]) for i in range(n_points)]


def walk_camera(points, s: float, vfov_deg: float = 60.0) -> Camera:
    """Camera at fraction s in [0, 1) of the path, looking ahead and down
    (0.15 below the point half a segment further along)."""
    umax = len(points) - 3.0
    u = s * (umax - 0.5)
    p = _catmull_rom(points, u)
    q = _catmull_rom(points, u + 0.5)
    target = q + np.array([0.0, -0.15, 0.0])
    return camera_look_at(p, target, [0, 1, 0], vfov_deg)


SERVED_RESOLUTIONS = [(512, 512), (1280, 720), (1920, 1080), (3840, 2160)]


def served_trace(seed: int, rate: float, duration: float, path_seed: int | None = None):
    """Render requests for a served run: Poisson arrivals at ``rate`` per
    second over ``duration`` seconds, resolution uniform over 512^2, 720p,
    1080p, 4K, K uniform in 3..8, cameras along a walk-through spline in
    arrival order.  Draw order: inter-arrival gaps (drawn until the duration
    is covered), then resolution index and K per request.
    Returns a list of (arrival_s, Camera, W, H, K)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    arrivals = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        arrivals.append(t)
    n = len(arrivals)
    ri = rng.integers(0, len(SERVED_RESOLUTIONS), size=n)
    ks = rng.integers(3, 9, size=n)
    pts = spline_path(seed + 1 if path_seed is None else path_seed)
    out = []
    for i, a in enumerate(arrivals):
        W, H = SERVED_RESOLUTIONS[int(ri[i])]
        out.append((a, walk_camera(pts, i / max(n, 1)), W, H, int(ks[i])))
    return out
