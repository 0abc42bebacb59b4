"""Seeded synthetic inputs: editable-Gaussian scenes, cameras and targets.

This module only draws inputs.  It holds none of the rasterizer's arithmetic
(no projection, shading, sorting or compositing), so both the HIP path and the
CPU oracle can consume exactly the same arrays.

Scenes stand in for the paper's volume datasets (§5.1, Table 1), which are not
available: each basic model is a set of editable Gaussians with the attributes
of §4.3 (geometry mu, q, s, o, n and shading delta-c, k_a, k_d, k_s, beta) and
a per-model palette colour c_p (§4.3).  Isosurface-shaped means mimic the
nested shells that the paper's basic transfer functions extract (§4, Fig. 1),
and composed scenes concatenate several such models (§4.5).

Array layout: every attribute is a float32 plane of shape [k, n]
(component-major, "SoA"):
    mean[3,n]  log_scale[3,n]  quat[4,n] (w,x,y,z)  opacity[1,n]
    normal[3,n]  color[3,n]  shade[4,n] (k_a, k_d, k_s, beta)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PLANES = ("mean", "log_scale", "quat", "opacity", "normal", "color", "shade")
PLANE_DIMS = {"mean": 3, "log_scale": 3, "quat": 4, "opacity": 1,
              "normal": 3, "color": 3, "shade": 4}

# Seed bases per workload: scene, target, camera; model m adds 100*m.
SEED_SCENE, SEED_TARGET, SEED_CAMERA = 1000, 2000, 3000


@dataclass
class Model:
    """One basic model: SoA planes plus its palette colour c_p."""
    planes: dict
    palette: np.ndarray            # (3,) float32, mean of the drawn base colours
    base: np.ndarray = None        # (3, n) float32, the drawn base colours

    @property
    def n(self) -> int:
        return int(self.planes["mean"].shape[1])


@dataclass
class Edit:
    """Per-model edit row (§4.5): recolour, opacity scale, light-magnitude
    transform lambda*k + b on (k_a, k_d, k_s, beta), and the light."""
    palette: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))
    opacity_scale: float = 1.0
    shade_scale: np.ndarray = field(default_factory=lambda: np.ones(4, np.float32))
    shade_bias: np.ndarray = field(default_factory=lambda: np.zeros(4, np.float32))
    light_dir: np.ndarray = field(default_factory=lambda: np.array([0, 0, 1], np.float32))
    headlight: bool = True

    def row(self) -> np.ndarray:
        """16 float32 words: palette[3], opacity_scale, shade_scale[4],
        shade_bias[4], light_dir[3], headlight (stored as int32 bits)."""
        r = np.zeros(16, np.float32)
        r[0:3] = self.palette
        r[3] = self.opacity_scale
        r[4:8] = self.shade_scale
        r[8:12] = self.shade_bias
        r[12:15] = self.light_dir
        r.view(np.int32)[15] = 1 if self.headlight else 0
        return r


def identity_edit(model: Model) -> Edit:
    return Edit(palette=model.palette.copy())


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).
    R (3x3, world->camera, row-major) and t map x_cam = R x_world + t."""
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def row(self) -> np.ndarray:
        """16 float32 words: R[9] row-major, t[3], fx, fy, cx, cy."""
        return np.concatenate([self.R.reshape(-1), self.t,
                               [self.fx, self.fy, self.cx, self.cy]]).astype(np.float32)

    @property
    def center(self) -> np.ndarray:
        return (-self.R.astype(np.float64).T @ self.t.astype(np.float64))


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------
def look_at(eye, target=(0.0, 0.0, 0.0), width=128, height=128, fov_deg=40.0,
            up=(0.0, 0.0, 1.0)) -> Camera:
    """Camera at `eye` looking at `target`; world up +z (+y if the view
    direction is parallel to z).  fx = fy = (W/2)/tan(FOV/2), principal point
    at the image centre; pixel (i, j) has its centre at (i+0.5, j+0.5)."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    f = target - eye
    f /= np.linalg.norm(f)
    up = np.asarray(up, np.float64)
    if abs(float(np.dot(f, up))) > 1.0 - 1e-9:
        up = np.array([0.0, 1.0, 0.0])
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f]).astype(np.float64)
    t = -R @ eye
    focal = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Camera(R.astype(np.float32), t.astype(np.float32), np.float32(focal),
                  np.float32(focal), np.float32(width / 2.0), np.float32(height / 2.0),
                  width, height)


def fibonacci_sphere(n: int, radius: float = 4.0) -> np.ndarray:
    """n points on a sphere: z_i = 1 - 2(i+1/2)/n, golden-angle azimuth."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - 2.0 * (i + 0.5) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def uniform_sphere(n: int, seed: int, radius: float = 4.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return radius * v


def orbit(n: int, elevation_deg: float = 20.0, step_deg: float = 6.0,
          radius: float = 4.0) -> np.ndarray:
    el = math.radians(elevation_deg)
    az = np.radians(step_deg * np.arange(n))
    return radius * np.stack([math.cos(el) * np.cos(az), math.cos(el) * np.sin(az),
                              np.full(n, math.sin(el))], axis=1)


def cameras_at(eyes, width, height, fov_deg=40.0):
    return [look_at(e, width=width, height=height, fov_deg=fov_deg) for e in eyes]


def camera_table(cams) -> np.ndarray:
    return np.stack([c.row() for c in cams]).astype(np.float32)


# ----------------------------------------------------------------------------
# Gaussian attributes
# ----------------------------------------------------------------------------
def _unit(rng, n, d):
    v = rng.normal(size=(d, n))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    return v


def attributes(means: np.ndarray, rng, log_scale_mu=-4.0, log_scale_sigma=0.5) -> Model:
    """Attribute distributions of the synthetic configs: log-scales
    N(mu, sigma) per axis, uniform unit quaternions, opacity sigmoid(N(0,1)),
    base colour U(0,1)^3, uniform unit normals, (k_a, k_d, k_s, beta) U(0,1).
    The palette c_p is the mean base colour and color = delta-c = base - c_p."""
    n = means.shape[1]
    log_scale = rng.normal(log_scale_mu, log_scale_sigma, size=(3, n))
    quat = _unit(rng, n, 4)
    opacity = 1.0 / (1.0 + np.exp(-rng.normal(size=(1, n))))
    base = rng.uniform(0.0, 1.0, size=(3, n))
    normal = _unit(rng, n, 3)
    shade = rng.uniform(0.0, 1.0, size=(4, n))
    palette = base.mean(axis=1).astype(np.float32)
    delta = base.astype(np.float32) - palette[:, None]
    planes = {
        "mean": means.astype(np.float32), "log_scale": log_scale.astype(np.float32),
        "quat": quat.astype(np.float32), "opacity": opacity.astype(np.float32),
        "normal": normal.astype(np.float32), "color": delta.astype(np.float32),
        "shade": shade.astype(np.float32),
    }
    return Model({k: np.ascontiguousarray(v) for k, v in planes.items()}, palette,
                 np.ascontiguousarray(base.astype(np.float32)))


def plain_planes(model: Model) -> dict:
    """Render-ready planes of the plain method (one basic model, no edits):
    the colour plane is the drawn base colour itself."""
    out = dict(model.planes)
    out["color"] = model.base
    return out


def uniform_means(n: int, rng) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=(3, n))


class ScalarField:
    """Synthetic scalar field: min of a noisy sphere and two tori.
    f_sph = |x| - 0.6 (1 + 0.1 eta(x/|x|)), eta a normalised sum of 4 seeded
    random-phase sinusoids; tori of radii (0.75, 0.12) in the xy and xz planes."""

    def __init__(self, seed: int):
        rng = np.random.default_rng(seed)
        d = rng.normal(size=(4, 3))
        self.dirs = d / np.linalg.norm(d, axis=1, keepdims=True)
        self.freq = rng.uniform(2.0, 6.0, size=4)
        self.amp = rng.uniform(0.5, 1.0, size=4)
        self.phase = rng.uniform(0.0, 2 * math.pi, size=4)

    def __call__(self, p: np.ndarray) -> np.ndarray:      # p: (m, 3)
        r = np.linalg.norm(p, axis=1)
        u = p / np.maximum(r, 1e-12)[:, None]
        eta = (self.amp[None, :] * np.sin(self.freq[None, :] * (u @ self.dirs.T)
                                          + self.phase[None, :])).sum(1) / self.amp.sum()
        f_sph = r - 0.6 * (1.0 + 0.1 * eta)
        x, y, z = p[:, 0], p[:, 1], p[:, 2]
        R_, r_ = 0.75, 0.12
        f_t1 = np.sqrt((np.sqrt(x * x + y * y) - R_) ** 2 + z * z) - r_
        f_t2 = np.sqrt((np.sqrt(x * x + z * z) - R_) ** 2 + y * y) - r_
        return np.minimum(f_sph, np.minimum(f_t1, f_t2))


def isosurface_means(n: int, rng, field_seed: int, level: float = 0.0,
                     width: float = 0.01, grid: int = 128) -> np.ndarray:
    """Rejection-sample n means uniformly in {x in [-1,1]^3 : |f(x) - level| < width}.

    Candidates are drawn uniformly from the grid cells that can meet the
    band: away from the origin f is Lipschitz with constant < 2.5 (tori: 1;
    noisy sphere: 1 + 0.36/|x|), so a cell whose centre value is farther than
    width + 2.5 * half-diagonal from the level cannot; cells near the origin
    are always kept.  Uniform over a superset plus rejection is uniform over
    the band."""
    fld = ScalarField(field_seed)
    h = 2.0 / grid
    c = (np.arange(grid) + 0.5) * h - 1.0
    centres = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    reach = 2.5 * h * math.sqrt(3.0) / 2.0
    near0 = np.linalg.norm(centres, axis=1) < 0.3 + h
    cells = centres[(np.abs(fld(centres) - level) <= width + reach) | near0]
    out, have = [], 0
    while have < n:
        m = max(8 * (n - have), 1 << 16)
        p = cells[rng.integers(0, cells.shape[0], m)] + rng.uniform(-h / 2, h / 2, size=(m, 3))
        keep = p[np.abs(fld(p) - level) < width]
        out.append(keep)
        have += keep.shape[0]
    return np.concatenate(out)[:n].T.copy()


# ----------------------------------------------------------------------------
# workloads (the five synthetic configurations)
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    models: list
    edits: list
    cameras: list
    width: int
    height: int
    targets_seed: int


def small_scene(n: int, seed: int, log_scale_mu=-4.0, log_scale_sigma=0.5) -> Model:
    rng = np.random.default_rng(seed)
    return attributes(uniform_means(n, rng), rng, log_scale_mu, log_scale_sigma)


def c1(seed_offset: int = 0) -> Workload:
    """One model of 10k uniform Gaussians, one 128x128 camera at radius 4."""
    m = small_scene(10_000, SEED_SCENE + 1 + seed_offset)
    cam = look_at((0.0, -4.0, 0.0), width=128, height=128)
    return Workload("c1-uniform-10k-128px", [m], [identity_edit(m)], [cam], 128, 128,
                    SEED_TARGET + 1)


def isosurface_model(n: int, seed: int, level: float = 0.0, field_seed: int = SEED_SCENE + 2):
    rng = np.random.default_rng(seed)
    return attributes(isosurface_means(n, rng, field_seed, level), rng)


def c2(n: int = 300_000, n_views: int = 100, width: int = 800) -> Workload:
    """One isosurface model, Fibonacci cameras at radius 4, 800x800."""
    m = isosurface_model(n, SEED_SCENE + 2)
    cams = cameras_at(fibonacci_sphere(n_views), width, width)
    return Workload(f"c2-isosurface-{n}-{width}px", [m], [identity_edit(m)], cams,
                    width, width, SEED_TARGET + 2)


def c3_edits(models, seed: int):
    rng = np.random.default_rng(seed)
    edits = []
    for _m in models:
        s = float(rng.uniform(0.5, 1.5))
        d = rng.normal(size=3)
        edits.append(Edit(palette=rng.uniform(0, 1, 3).astype(np.float32),
                          opacity_scale=float(rng.uniform(0.0, 2.0)),
                          shade_scale=np.array([s, s, s, 1.0], np.float32),
                          shade_bias=np.zeros(4, np.float32),
                          light_dir=(d / np.linalg.norm(d)).astype(np.float32),
                          headlight=False))
    return edits


def c3(n_per: int = 150_000, k: int = 8, n_views: int = 60, width: int = 1024) -> Workload:
    """k nested-shell models at levels -0.25 + 0.07 m, edited and composed."""
    models = [isosurface_model(n_per, SEED_SCENE + 3 + 100 * m, -0.25 + 0.07 * m)
              for m in range(k)]
    cams = cameras_at(orbit(n_views), width, width)
    return Workload(f"c3-compose-{k}x{n_per}-{width}px", models,
                    c3_edits(models, SEED_SCENE + 3 + 7), cams, width, width,
                    SEED_TARGET + 3)


def c4(sizes=(50_000, 120_000, 250_000, 500_000), levels=(-0.1, 0.0, 0.1, 0.2),
       n_views: int = 32, width: int = 800) -> Workload:
    models = [isosurface_model(s, SEED_SCENE + 4 + 100 * m, lv)
              for m, (s, lv) in enumerate(zip(sizes, levels))]
    cams = cameras_at(fibonacci_sphere(n_views), width, width)
    return Workload(f"c4-batched-{len(sizes)}models-{n_views}views-{width}px", models,
                    [identity_edit(m) for m in models], cams, width, width,
                    SEED_TARGET + 4)


def c5_views(n_train=200, n_test=60, width=1024):
    train = cameras_at(uniform_sphere(n_train, 5000), width, width)
    test = cameras_at(uniform_sphere(n_test, 5001), width, width)
    return train, test


def random_target(n_views: int, height: int, width: int, seed: int) -> np.ndarray:
    """Random RGBA target image U(0,1), layout [views, 4, H, W]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n_views, 4, height, width)).astype(np.float32)


def view_maps(height: int, width: int, seed: int, n_gauss: int = 257) -> dict:
    """Seeded float32 maps of one view for the training regularisers: the
    alpha-weighted depth of a smooth bumpy surface (depth 2.7-3.5), an alpha
    map near 0.95 with a hole that drops below 0.5, normals N(0, 1) per
    component, offset colours U(-0.5, 0.5), shading terms and a target colour
    U(0, 1), and opacities U(-0.2, 1.5) (negative values reach the L1's
    sign)."""
    rng = np.random.default_rng(seed)
    ys, xs = np.meshgrid(np.arange(height) + 0.5, np.arange(width) + 0.5, indexing="ij")
    u, v = xs / width, ys / height
    d = 3.0 + 0.3 * np.sin(5 * u + 1.0) * np.cos(4 * v) + 0.2 * u * v
    alpha = np.clip(0.95 - 0.9 * np.exp(-((u - 0.6) ** 2 + (v - 0.4) ** 2) / 0.01), 0.0, 1.0)
    f = np.float32
    return {"depth": (d * alpha).astype(f), "alpha": alpha.astype(f),
            "normal": rng.normal(size=(3, height, width)).astype(f),
            "delta_c": rng.uniform(-0.5, 0.5, (3, height, width)).astype(f),
            "shade": rng.uniform(0, 1, (4, height, width)).astype(f),
            "target": rng.uniform(0, 1, (3, height, width)).astype(f),
            "opacity": rng.uniform(-0.2, 1.5, n_gauss).astype(f)}
