"""Seeded synthetic scenes and cameras shaped like the paper's workloads.

This module only draws random numbers and fills parameter records; it holds
none of the renderer's arithmetic, so the GPU path and the FP64 oracle can
both take their inputs from it.

Scene layout (structure of arrays, float32, host numpy):
  mean    [3, N]      world-space centre
  scale   [3, N]      linear standard deviations along the local axes
  quat    [4, N]      (r, i, j, k), not necessarily unit
  opacity [N]         opacity coefficient sigma in (0, 1)
  sh      [K*3, N]    SH coefficients, row (k*3 + channel), K = (deg+1)^2

Camera record (dict): model ('pinhole' | 'equidistant' | 'kb'), width, height
of the BEAP grid, native intrinsics fx, fy, cx, cy, k (4 distortion
coefficients), BEAP angular extents fov_x, fov_y (radians), and the
world-to-camera pose R (3x3), t (3) with x_cam = R x_world + t (OpenCV axes:
x right, y down, z forward).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SH_C0 = 0.28209479177387814  # DC basis value, used only to encode a target RGB


@dataclass
class Scene:
    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def arrays(self):
        return self.mean, self.scale, self.quat, self.opacity, self.sh

    def copy(self) -> "Scene":
        return Scene(self.mean.copy(), self.scale.copy(), self.quat.copy(),
                     self.opacity.copy(), self.sh.copy(), self.sh_degree)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.mean[:, idx]), np.ascontiguousarray(self.scale[:, idx]),
                     np.ascontiguousarray(self.quat[:, idx]), np.ascontiguousarray(self.opacity[idx]),
                     np.ascontiguousarray(self.sh[:, idx]), self.sh_degree)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Haar-uniform rotation: QR of a 3x3 Gaussian matrix with the sign of R's
    diagonal folded into Q, then a reflection fixed to det +1."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def scene_small(n: int = 1000, seed: int = 0) -> Scene:
    """Plain-forward scene: x, y ~ U[-1, 1], z ~ U[2, 6]; scales log-U[0.02, 0.2];
    unit-quaternion rotations; opacity U[0.1, 0.9]; RGB U[0, 1] as SH degree 0."""
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)])
    scale = np.exp(rng.uniform(math.log(0.02), math.log(0.2), (3, n)))
    quat = rng.standard_normal((4, n))
    quat /= np.linalg.norm(quat, axis=0, keepdims=True)
    opacity = rng.uniform(0.1, 0.9, n)
    rgb = rng.uniform(0, 1, (3, n))
    sh = (rgb - 0.5) / SH_C0
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), 0)


def scene_box(n: int, seed: int = 0, half: float = 10.0, smin: float = 0.01, smax: float = 0.5,
              sh_degree: int = 3, sh_std: float = 0.3) -> Scene:
    """Large-scene generator: means uniform in a (2*half)^3 box around the origin,
    scales log-uniform [smin, smax], SH coefficients ~ N(0, sh_std^2),
    opacity U[0.1, 0.9], uniform rotations."""
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-half, half, (3, n))
    scale = np.exp(rng.uniform(math.log(smin), math.log(smax), (3, n)))
    quat = rng.standard_normal((4, n))
    quat /= np.linalg.norm(quat, axis=0, keepdims=True)
    opacity = rng.uniform(0.1, 0.9, n)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, sh_std, (k * 3, n))
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), sh_degree)


def scene_slice(n: int = 200, seed: int = 0) -> Scene:
    """Finite-difference slice: the large-scene generator restricted to
    [-1.5, 1.5]^2 x [1, 4] m."""
    s = scene_box(n, seed)
    rng = np.random.default_rng(seed + 7919)
    s.mean[0] = rng.uniform(-1.5, 1.5, n).astype(np.float32)
    s.mean[1] = rng.uniform(-1.5, 1.5, n).astype(np.float32)
    s.mean[2] = rng.uniform(1.0, 4.0, n).astype(np.float32)
    return s


def perturb(scene: Scene, seed: int) -> Scene:
    """Target-scene perturbation: mean += N(0, 0.01^2); log scale += N(0, 0.05^2);
    quat += N(0, 0.02^2) then renormalised; opacity += N(0, 0.02^2) clipped to
    [0.01, 0.99]; SH += N(0, 0.02^2)."""
    rng = np.random.default_rng(seed)
    n = scene.n
    q = scene.quat.astype(np.float64) + rng.normal(0, 0.02, (4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return Scene(
        _f32(scene.mean + rng.normal(0, 0.01, (3, n))),
        _f32(np.exp(np.log(scene.scale.astype(np.float64)) + rng.normal(0, 0.05, (3, n)))),
        _f32(q),
        _f32(np.clip(scene.opacity + rng.normal(0, 0.02, n), 0.01, 0.99)),
        _f32(scene.sh + rng.normal(0, 0.02, scene.sh.shape)),
        scene.sh_degree,
    )


def _pose(R=None, position=None):
    R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64)
    c = np.zeros(3) if position is None else np.asarray(position, dtype=np.float64)
    return R, -R @ c


def camera_pinhole(width: int, height: int, fov_x_deg: float, R=None, position=None) -> dict:
    """Pinhole camera with horizontal FoV; the BEAP grid spans the same angular
    box as the native sensor (vertical FoV from the focal length)."""
    f = (width / 2) / math.tan(math.radians(fov_x_deg) / 2)
    Rw, t = _pose(R, position)
    return dict(model="pinhole", width=width, height=height, fx=f, fy=f, cx=width / 2, cy=height / 2,
                k=[0.0, 0.0, 0.0, 0.0], fov_x=math.radians(fov_x_deg),
                fov_y=2 * math.atan((height / 2) / f), R=Rw, t=t)


def camera_pinhole_native(width: int, height: int, fov_x_deg: float, R=None, position=None,
                          principal=(0.5, 0.5), aspect: float = 1.0) -> dict:
    """Pinhole camera rendered on its own pixel grid (one ray per native
    pixel); the principal point at the given fractions of the sensor and
    fy = aspect * fx.  fov_x / fov_y record the sensor's angular extent."""
    f = (width / 2) / math.tan(math.radians(fov_x_deg) / 2)
    Rw, t = _pose(R, position)
    cx, cy = principal[0] * width, principal[1] * height
    fy = aspect * f
    return dict(model="pinhole", grid="native", width=width, height=height, fx=f, fy=fy, cx=cx, cy=cy,
                k=[0.0, 0.0, 0.0, 0.0], fov_x=math.atan(cx / f) + math.atan((width - cx) / f),
                fov_y=math.atan(cy / fy) + math.atan((height - cy) / fy), R=Rw, t=t)


def camera_equidistant(width: int, height: int, fov_deg: float, R=None, position=None) -> dict:
    """Equidistant fisheye (Kannala-Brandt with zero distortion). The BEAP grid
    has equal angular pitch along both axes."""
    fov = math.radians(fov_deg)
    f = (width / 2) / (fov / 2)
    Rw, t = _pose(R, position)
    return dict(model="equidistant", width=width, height=height, fx=f, fy=f, cx=width / 2, cy=height / 2,
                k=[0.0, 0.0, 0.0, 0.0], fov_x=fov, fov_y=fov * height / width, R=Rw, t=t)


def kb_coeffs(seed: int, fov_deg: float, lim: float = 0.05) -> list:
    """Distortion coefficients k1..k4 ~ U[-lim, lim], re-drawn (seeded) until the
    distorted angle theta*(1 + k1 theta^2 + ... + k4 theta^8) is strictly
    increasing on [0, fov/2]."""
    rng = np.random.default_rng(seed)
    th = np.linspace(0.0, math.radians(fov_deg) / 2, 2048)
    while True:
        k = rng.uniform(-lim, lim, 4)
        td = th * (1 + k[0] * th**2 + k[1] * th**4 + k[2] * th**6 + k[3] * th**8)
        if np.all(np.diff(td) > 0):
            return [float(x) for x in k]


def camera_kb(width: int, height: int, fov_deg: float, seed: int = 0, R=None, position=None,
              fov_y_deg: float | None = None) -> dict:
    """Kannala-Brandt fisheye with random k1..k4; the focal length maps the
    half-FoV to the sensor's horizontal edge; BEAP grid with equal pitch
    unless a vertical FoV is given."""
    k = kb_coeffs(seed, fov_deg)
    th = math.radians(fov_deg) / 2
    td = th * (1 + k[0] * th**2 + k[1] * th**4 + k[2] * th**6 + k[3] * th**8)
    f = (width / 2) / td
    fov = math.radians(fov_deg)
    Rw, t = _pose(R, position)
    fov_y = math.radians(fov_y_deg) if fov_y_deg is not None else fov * height / width
    return dict(model="kb", width=width, height=height, fx=f, fy=f, cx=width / 2, cy=height / 2,
                k=k, fov_x=fov, fov_y=fov_y, R=Rw, t=t)


def camera_slice(seed: int = 0, res: int = 32) -> dict:
    """Finite-difference slice camera: Kannala-Brandt 190 deg on a res x res
    BEAP grid spanning 190 x 142.5 degrees (the 1280 x 960 frame's extents)."""
    return camera_kb(res, res, 190.0, seed=seed, fov_y_deg=142.5)


def random_pose(rng: np.random.Generator, half: float = 8.0):
    return random_rotation(rng), rng.uniform(-half, half, 3)


# ---------------------------------------------------------------- workloads --

def workload_small(seed: int = 0):
    """1,000 Gaussians SH0, pinhole 60 deg, 64x64 BEAP grid."""
    return scene_small(1000, seed), [camera_pinhole(64, 64, 60.0)]


def workload_fisheye_forward(seed: int = 0, n: int = 100_000, width: int = 1024):
    """100k Gaussians SH3 in a 20 m box, equidistant fisheye 180 deg, 1024x1024 BEAP grid."""
    return scene_box(n, seed), [camera_equidistant(width, width, 180.0)]


def workload_kb_train(seed: int = 0, n: int = 500_000, width: int = 1280, height: int = 960):
    """500k Gaussians SH3, Kannala-Brandt 190 deg fisheye 1280x960; the target is
    rendered from perturbed parameters."""
    scene = scene_box(n, seed)
    return scene, [camera_kb(width, height, 190.0, seed=seed)], perturb(scene, seed + 1)


def workload_serving_requests(count: int, seed: int = 0):
    """Request cameras in thirds: pinhole 60 deg 640x480, equidistant 180 deg
    1024x1024 and KB 200 deg 1920x1080, random poses within the scene box."""
    rng = np.random.default_rng(seed)
    cams = []
    for r in range(count):
        R, c = random_pose(rng)
        kind = r % 3
        if kind == 0:
            cams.append(camera_pinhole(640, 480, 60.0, R, c))
        elif kind == 1:
            cams.append(camera_equidistant(1024, 1024, 180.0, R, c))
        else:
            cams.append(camera_kb(1920, 1080, 200.0, seed=seed + r, R=R, position=c))
    return cams


def workload_batched_views(seed: int = 0, width: int = 1920, height: int = 1080):
    """Eight 1920x1080 views: four pinhole (90 deg horizontal) and four
    equidistant 180 deg, random poses."""
    rng = np.random.default_rng(seed)
    cams = []
    for v in range(8):
        R, c = random_pose(rng)
        if v < 4:
            cams.append(camera_pinhole(width, height, 90.0, R, c))
        else:
            cams.append(camera_equidistant(width, height, 180.0, R, c))
    return cams
