"""FP64 oracle for the exact Gaussian ray renderer (3DGEER, arXiv 2505.24053).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never loads it; it shares no code with ``paper_2505_24053_amd``
except the seeded input generators of ``paper_2505_24053_amd.synth``.

The heavy lifting is in ``geer_oracle.c`` (plain C, FP64, brute force over
every ray-Gaussian pair, OpenMP over rays).  This module compiles it with gcc
on first use, marshals arguments, and adds the pieces that are easiest to
state with library primitives:

* ``tile_list``: the (tile, depth key, index) ordering of the association
  list, done with ``numpy.lexsort`` (the paper's global sort by
  FrustumID + depth, Alg. 1);
* ``valid_mask``: BEAP rays that land on the native sensor through the
  pinhole or Kannala-Brandt projection (App. E).

Every function here follows the passage cited in its docstring.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "geer_oracle.c")
LIB = os.path.join(HERE, "libgeer_oracle.so")

MODELS = {"pinhole": 0, "equidistant": 1, "kb": 2}
DEFAULT_OPTS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, lambda_mode=0, lambda_fixed=3.0, splat=False)


class View(C.Structure):
    _fields_ = [("model", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("grid", C.c_int32),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("k", C.c_double * 4), ("fov_x", C.c_double), ("fov_y", C.c_double),
                ("R", C.c_double * 9), ("t", C.c_double * 3)]


class Opts(C.Structure):
    _fields_ = [("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double),
                ("lambda_fixed", C.c_double), ("lambda_mode", C.c_int32), ("splat", C.c_int32)]


class SceneC(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("pad_", C.c_int32),
                ("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


ASSOC_DT = np.dtype([("hx0", np.int32), ("hx1", np.int32), ("hy0", np.int32), ("hy1", np.int32),
                     ("count", np.uint32), ("key", np.uint32), ("culled", np.int32), ("pad_", np.int32)])

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no fused multiply-add, no fast math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
                               "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(LIB)
            P = C.POINTER
            L.orc_assoc_fp32.argtypes = [P(SceneC), P(View), P(Opts), C.c_void_p]
            L.orc_render.argtypes = [P(SceneC), P(View), P(Opts), C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_void_p, C.c_int]
            L.orc_render_backward.argtypes = [P(SceneC), P(View), P(Opts), C.c_int64, C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_int]
            L.orc_sh_basis.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
            L.orc_pair.argtypes = [P(SceneC), P(View), P(Opts), C.c_int64, C.c_void_p, C.c_void_p]
            L.orc_edges.argtypes = [P(View), C.c_void_p, C.c_void_p, P(C.c_int), P(C.c_int)]
            L.orc_lambda2_hat.argtypes = [C.c_float, C.c_float, C.c_int, C.c_double]
            L.orc_lambda2_hat.restype = C.c_float
            L.orc_contrib_mask.argtypes = [P(SceneC), P(View), P(Opts), C.c_int64, C.c_void_p, C.c_void_p]
            L.orc_tile_pairs_contribute.argtypes = [P(SceneC), P(View), P(Opts), C.c_int64, C.c_void_p, C.c_void_p,
                                                    C.c_void_p, C.c_int]
            _lib = L
    return _lib


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def make_view(cam: dict) -> View:
    v = View()
    v.model = MODELS[cam["model"]]
    v.width, v.height = int(cam["width"]), int(cam["height"])
    v.grid = 1 if cam.get("grid", "beap") == "native" else 0
    v.fx, v.fy, v.cx, v.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    for i in range(4):
        v.k[i] = float(cam["k"][i])
    v.fov_x, v.fov_y = float(cam["fov_x"]), float(cam["fov_y"])
    R = np.asarray(cam["R"], dtype=np.float64).reshape(9)
    t = np.asarray(cam["t"], dtype=np.float64).reshape(3)
    for i in range(9):
        v.R[i] = R[i]
    for i in range(3):
        v.t[i] = t[i]
    return v


def make_opts(**kw) -> Opts:
    d = dict(DEFAULT_OPTS)
    d.update(kw)
    o = Opts()
    o.alpha_min, o.alpha_max, o.t_min = float(d["alpha_min"]), float(d["alpha_max"]), float(d["t_min"])
    o.lambda_fixed, o.lambda_mode = float(d["lambda_fixed"]), int(d["lambda_mode"])
    o.splat = 1 if d["splat"] else 0
    return o


class _SceneRef:
    """Keeps contiguous FP64 copies (exact for FP32 inputs) alive while C
    holds their pointers."""

    def __init__(self, scene):
        self.arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in scene.arrays()]
        s = SceneC()
        s.n = scene.n
        s.sh_degree = scene.sh_degree
        s.mean, s.scale, s.quat, s.opacity, s.sh = (a.ctypes.data for a in self.arrs)
        self.c = s


def assoc_fp32(scene, cam, **opts):
    """FP32 association reference (particle bounding frustum against the
    camera sub-frusta, Sec. 3.2 / App. D): per Gaussian the half-tile
    rectangle, tile count, depth key and 3-sigma cull flag."""
    L = lib()
    ref = _SceneRef(scene)
    out = np.zeros(scene.n, dtype=ASSOC_DT)
    L.orc_assoc_fp32(C.byref(ref.c), C.byref(make_view(cam)), C.byref(make_opts(**opts)), _ptr(out))
    return out


def tile_grid(cam):
    tw = (int(cam["width"]) + 15) // 16
    th = (int(cam["height"]) + 15) // 16
    return tw, th


def tile_list(assoc, cam):
    """Expand each visible Gaussian to every 16x16 tile of its rectangle and
    order the entries by (tile id, depth key, Gaussian index) -- the
    DuplicateWithKeys / SortByKeys / IdentifyFrustumRanges steps of Alg. 1.
    Returns (tile ids, Gaussian ids, ranges[ntiles + 1])."""
    tw, th = tile_grid(cam)
    vis = np.nonzero(assoc["count"] > 0)[0]
    a = assoc[vis]
    tx0, tx1 = a["hx0"].astype(np.int64) // 2, a["hx1"].astype(np.int64) // 2
    ty0, ty1 = a["hy0"].astype(np.int64) // 2, a["hy1"].astype(np.int64) // 2
    wt = tx1 - tx0 + 1
    cnt = wt * (ty1 - ty0 + 1)
    assert np.all(cnt == a["count"].astype(np.int64))
    total = int(cnt.sum())
    owner = np.repeat(np.arange(vis.size), cnt)
    local = np.arange(total) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    tiles = (ty0[owner] + local // wt[owner]) * tw + tx0[owner] + local % wt[owner]
    gids = vis[owner].astype(np.int64)
    keys = a["key"][owner].astype(np.uint64)
    order = np.lexsort((gids, keys, tiles))
    tiles, gids = tiles[order], gids[order]
    ranges = np.searchsorted(tiles, np.arange(tw * th + 1), side="left")
    return tiles, gids, ranges


MAX_BRANCHES = 64


def render(scene, cam, pix=None, nthreads: int = 0, branches: bool = True, **opts):
    """Brute-force FP64 render of BEAP pixels (all when ``pix`` is None),
    front-to-back compositing of Eq. color with the contribution rule of
    Sec. 3.2.  Returns dict(rgb [P,3], depth [P], trans [P], ncomp [P],
    amb [P], pix) from the FP64 decisions; ``amb`` marks rays on which some
    decision (a contribution threshold, or the termination test) lies within
    the FP32 error band, so FP32 may take another branch.

    With ``branches`` every flagged ray's alternative outcomes are listed:
    ``branch_idx`` (positions in ``pix`` of the flagged rays),
    ``branch_leaves`` [F, MAX_BRANCHES, 5] = (r, g, b, depth, T) of each
    decision sequence and ``branch_count`` [F] (above MAX_BRANCHES: too many
    to list)."""
    L = lib()
    w, h = int(cam["width"]), int(cam["height"])
    if pix is None:
        pix = np.arange(w * h, dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    ref = _SceneRef(scene)
    view, op = make_view(cam), make_opts(**opts)

    def run(p, with_leaves):
        n = p.size
        out = dict(rgb=np.zeros((n, 3)), depth=np.zeros(n), trans=np.zeros(n), ncomp=np.zeros(n, np.int32),
                   amb=np.zeros(n, np.int32))
        leaves = np.zeros((n, MAX_BRANCHES, 5)) if with_leaves else None
        nleaves = np.zeros(n, np.int64) if with_leaves else None
        rc = L.orc_render(C.byref(ref.c), C.byref(view), C.byref(op), n, _ptr(p), _ptr(out["rgb"]),
                          _ptr(out["depth"]), _ptr(out["trans"]), _ptr(out["ncomp"]), _ptr(out["amb"]),
                          MAX_BRANCHES, _ptr(leaves), _ptr(nleaves), int(nthreads))
        if rc != 0:
            raise MemoryError("oracle render failed")
        return out, leaves, nleaves

    out, _, _ = run(pix, False)
    out["amb"] = out["amb"].astype(bool)
    out["pix"] = pix
    if branches:
        idx = np.nonzero(out["amb"])[0]
        if idx.size:
            _, leaves, nleaves = run(np.ascontiguousarray(pix[idx]), True)
        else:
            leaves, nleaves = np.zeros((0, MAX_BRANCHES, 5)), np.zeros(0, np.int64)
        out.update(branch_idx=idx, branch_leaves=leaves, branch_count=nleaves)
    return out


def branch_scores(got_rgb, got_depth, got_trans, ref, rgb_tol=2e-4, depth_rel=1e-3):
    """For each flagged ray of ``ref`` (a render with branches): the smallest,
    over its decision branches, of the largest gate ratio -- RGB and T
    max-abs over ``rgb_tol``, depth relative error over ``depth_rel``.  A
    score <= 1 means the values are one of the outcomes FP32 can produce.
    ``got_*`` are per-ray arrays aligned with ``ref["pix"]``.  Rays with more
    branches than listed score +inf."""
    idx = ref["branch_idx"]
    L = ref["branch_leaves"]
    cnt = ref["branch_count"]
    if idx.size == 0:
        return np.zeros(0)
    e_rgb = np.abs(np.asarray(got_rgb)[idx][:, None, :] - L[:, :, 0:3]).max(axis=2) / rgb_tol
    e_d = np.abs(np.asarray(got_depth)[idx][:, None] - L[:, :, 3]) / (1.0 + np.abs(L[:, :, 3])) / depth_rel
    e_t = np.abs(np.asarray(got_trans)[idx][:, None] - L[:, :, 4]) / rgb_tol
    score = np.maximum(np.maximum(e_rgb, e_d), e_t)
    listed = np.arange(L.shape[1])[None, :] < np.minimum(cnt, L.shape[1])[:, None]
    score = np.where(listed, score, np.inf).min(axis=1)
    return np.where(cnt > L.shape[1], np.inf, score)


def render_backward(scene, cam, pix, dl_drgb, nthreads: int = 0, **opts):
    """FP64 gradients of L (given dL/dRGB [P,3] on ``pix``) with respect to
    mean [3,N], scale [3,N], raw quaternion [4,N], opacity [N], SH [K*3,N]
    (App. C, with the corrected cross-product signs)."""
    L = lib()
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    g = np.ascontiguousarray(dl_drgb, dtype=np.float64).reshape(-1, 3)
    assert g.shape[0] == pix.size
    n = scene.n
    K = (scene.sh_degree + 1) ** 2
    out = dict(mean=np.zeros((3, n)), scale=np.zeros((3, n)), quat=np.zeros((4, n)), opacity=np.zeros(n),
               sh=np.zeros((K * 3, n)))
    ref = _SceneRef(scene)
    rc = L.orc_render_backward(C.byref(ref.c), C.byref(make_view(cam)), C.byref(make_opts(**opts)), pix.size,
                               _ptr(pix), _ptr(g), _ptr(out["mean"]), _ptr(out["scale"]), _ptr(out["quat"]),
                               _ptr(out["opacity"]), _ptr(out["sh"]), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle backward failed")
    return out


def contrib_mask(scene, cam, pix=None, **opts):
    """Brute-force [P, N] boolean mask of contributing (pixel, Gaussian) pairs
    under the contribution rule, without early termination (tiny inputs)."""
    w, h = int(cam["width"]), int(cam["height"])
    if pix is None:
        pix = np.arange(w * h, dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    mask = np.zeros((pix.size, scene.n), np.uint8)
    ref = _SceneRef(scene)
    lib().orc_contrib_mask(C.byref(ref.c), C.byref(make_view(cam)), C.byref(make_opts(**opts)), pix.size,
                           _ptr(pix), _ptr(mask))
    return mask.astype(bool)


def sh_basis(deg: int, dirs):
    """Real SH basis (Condon-Shortley phase) and its R^3 gradient at ``dirs``."""
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    K = (deg + 1) ** 2
    Y = np.zeros((d.shape[0], K))
    dY = np.zeros((d.shape[0], K, 3))
    lib().orc_sh_basis(deg, d.shape[0], _ptr(d), _ptr(Y), _ptr(dY))
    return Y, dY


def pair(scene, cam, g: int, d, with_band: bool = False, **opts):
    """(kappa, t*, sigma exp(-kappa/2), lambda_i^2) of one pair, FP64; with
    ``with_band`` also the FP32 error band of kappa that flags decisions."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(5)
    ref = _SceneRef(scene)
    lib().orc_pair(C.byref(ref.c), C.byref(make_view(cam)), C.byref(make_opts(**opts)), int(g), _ptr(d),
                   _ptr(out))
    return out if with_band else out[:4]


def edges(cam):
    """Half-tile edge tables: mirrored tan(theta/2) columns, tan(phi) rows."""
    w, h = int(cam["width"]), int(cam["height"])
    ex = np.zeros(w // 8 + 2, np.float32)
    ey = np.zeros(h // 8 + 2, np.float32)
    nx, ny = C.c_int(), C.c_int()
    lib().orc_edges(C.byref(make_view(cam)), _ptr(ex), _ptr(ey), C.byref(nx), C.byref(ny))
    return ex[:nx.value + 1], ey[:ny.value + 1]


def lambda2_hat(sigma: float, alpha_min: float = 1 / 255, mode: int = 0, lam_fixed: float = 3.0) -> float:
    return float(lib().orc_lambda2_hat(float(sigma), float(alpha_min), int(mode), float(lam_fixed)))


def pixel_dirs_camera(cam, pix):
    """FP64 camera-space unit directions of BEAP pixel centres (App. E); on
    a native pinhole grid the pixel's own ray, whose BEAP angles have the
    normalised image coordinates as tangents."""
    w, h = int(cam["width"]), int(cam["height"])
    pix = np.asarray(pix, dtype=np.int64)
    px, py = pix % w, pix // w
    if cam.get("grid", "beap") == "native":
        th = np.arctan((px + 0.5 - cam["cx"]) / cam["fx"])
        ph = np.arctan((py + 0.5 - cam["cy"]) / cam["fy"])
    else:
        th = -cam["fov_x"] / 2 + (px + 0.5) * cam["fov_x"] / w
        ph = -cam["fov_y"] / 2 + (py + 0.5) * cam["fov_y"] / h
    d = np.stack([np.sin(th) * np.cos(ph), np.cos(th) * np.sin(ph), np.cos(th) * np.cos(ph)], -1)
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def pixel_dirs_world(cam, pix):
    R = np.asarray(cam["R"], dtype=np.float64).reshape(3, 3)
    return pixel_dirs_camera(cam, pix) @ R


def valid_mask(cam):
    """BEAP rays whose native projection lands on the sensor (App. E).  The
    incidence angle is atan2(sqrt(x^2+y^2), z) so rays beyond 90 degrees are
    handled; pinhole rays need z > 0."""
    w, h = int(cam["width"]), int(cam["height"])
    if cam.get("grid", "beap") == "native":
        return np.ones((h, w), bool)  # the sensor's own pixels
    d = pixel_dirs_camera(cam, np.arange(w * h)).reshape(h, w, 3)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    rxy = np.hypot(x, y)
    if cam["model"] == "pinhole":
        with np.errstate(divide="ignore", invalid="ignore"):
            u = cam["fx"] * x / z + cam["cx"]
            v = cam["fy"] * y / z + cam["cy"]
        ok = z > 0
    else:
        inc = np.arctan2(rxy, z)
        k = cam["k"]
        td = inc * (1 + k[0] * inc**2 + k[1] * inc**4 + k[2] * inc**6 + k[3] * inc**8)
        with np.errstate(divide="ignore", invalid="ignore"):
            cx_ = np.where(rxy > 0, x / rxy, 0.0)
            cy_ = np.where(rxy > 0, y / rxy, 0.0)
        u = cam["fx"] * td * cx_ + cam["cx"]
        v = cam["fy"] * td * cy_ + cam["cy"]
        ok = np.ones_like(z, dtype=bool)
    return ok & (u >= 0) & (u < w) & (v >= 0) & (v < h)


def _distort(theta, k):
    t2 = theta * theta
    return theta * (1 + k[0] * t2 + k[1] * t2**2 + k[2] * t2**3 + k[3] * t2**4)


def kb_incidence(td, k):
    """Incidence angle theta of distorted radii td on the increasing branch of
    theta (1 + k1 theta^2 + ... + k4 theta^8) (App. E), by bisection to the
    last bit; NaN where td lies beyond that branch.  The branch ends at the
    first of 4096 even steps over [0, pi] where the derivative is <= 0."""
    td = np.asarray(td, dtype=np.float64)
    ts = np.pi * np.arange(1, 4097) / 4096
    t2 = ts * ts
    d = 1 + t2 * (3 * k[0] + t2 * (5 * k[1] + t2 * (7 * k[2] + t2 * 9 * k[3])))
    stop = np.nonzero(d <= 0)[0]
    hi_t = ts[stop[0]] if stop.size else np.pi
    lo = np.zeros_like(td)
    hi = np.full_like(td, hi_t)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        below = _distort(mid, k) < td
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    theta = 0.5 * (lo + hi)
    return np.where(td <= _distort(hi_t, k), theta, np.nan)


def reproject_positions(cam, native_size=None):
    """Continuous BEAP grid positions (x, y) of the native sensor's pixel
    centres (i + 1/2, j + 1/2) and whether a BEAP ray reaches them (App. E):
    the pinhole back-projection ((u - cx)/fx, (v - cy)/fy, 1), or the KB ray
    at incidence kb_incidence(|offset|) and the offset's azimuth; then
    theta = atan2(x, z), phi = atan(y / z), position = (angle + fov/2) n / fov
    - 1/2.  Positions more than half a pixel outside the grid are not
    reached."""
    w, h = int(cam["width"]), int(cam["height"])
    nw, nh = native_size if native_size else (w, h)
    jj, ii = np.mgrid[0:nh, 0:nw].astype(np.float64)
    mx = (ii + 0.5 - cam["cx"]) / cam["fx"]
    my = (jj + 0.5 - cam["cy"]) / cam["fy"]
    if cam["model"] == "pinhole":
        x, y, z = mx, my, np.ones_like(mx)
        ok = np.ones(mx.shape, bool)
    else:
        td = np.hypot(mx, my)
        th = kb_incidence(td, cam["k"])
        ok = np.isfinite(th)
        th = np.where(ok, th, 0.0)
        with np.errstate(invalid="ignore", divide="ignore"):
            x = np.where(td > 0, np.sin(th) * mx / td, 0.0)
            y = np.where(td > 0, np.sin(th) * my / td, 0.0)
        z = np.cos(th)
    tb = np.arctan2(x, z)
    with np.errstate(invalid="ignore", divide="ignore"):
        pb = np.where(z != 0, np.arctan(y / np.where(z != 0, z, 1.0)), np.sign(y) * np.pi / 2)
    gx = (tb + cam["fov_x"] / 2) * w / cam["fov_x"] - 0.5
    gy = (pb + cam["fov_y"] / 2) * h / cam["fov_y"] - 0.5
    ok &= (gx >= -0.5) & (gx <= w - 0.5) & (gy >= -0.5) & (gy <= h - 0.5)
    return gx, gy, ok


def reproject(cam, beap, native_size=None):
    """BEAP image [C, H, W] of `cam` resampled onto its native sensor
    (App. E inverse interpolation): at each reached native pixel the bilinear
    interpolation of the four BEAP pixels around its grid position (clamped
    into the grid), FP64; unreached pixels are 0.  Returns (native [C, Hn,
    Wn], valid [Hn, Wn])."""
    beap = np.asarray(beap, dtype=np.float64)
    C_, h, w = beap.shape
    gx, gy, ok = reproject_positions(cam, native_size)
    x = np.clip(np.where(ok, gx, 0.0), 0, w - 1)
    y = np.clip(np.where(ok, gy, 0.0), 0, h - 1)
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    x1 = np.minimum(x0 + 1, w - 1)
    y1 = np.minimum(y0 + 1, h - 1)
    fx, fy = x - x0, y - y0
    out = ((1 - fx) * (1 - fy) * beap[:, y0, x0] + fx * (1 - fy) * beap[:, y0, x1] +
           (1 - fx) * fy * beap[:, y1, x0] + fx * fy * beap[:, y1, x1])
    return np.where(ok[None], out, 0.0), ok


def _rotation(q):
    """Local-to-world rotations [N, 3, 3] of quaternions (r, i, j, k) [4, N]."""
    q = q / np.linalg.norm(q, axis=0, keepdims=True)
    r, i, j, k = q
    return np.stack([np.stack([1 - 2 * (j * j + k * k), 2 * (i * j - r * k), 2 * (i * k + r * j)], -1),
                     np.stack([2 * (i * j + r * k), 1 - 2 * (i * i + k * k), 2 * (j * k - r * i)], -1),
                     np.stack([2 * (i * k - r * j), 2 * (j * k + r * i), 1 - 2 * (i * i + j * j)], -1)], 1)


def _beap(x, y, z):
    th = np.arctan2(x, z)
    with np.errstate(divide="ignore", invalid="ignore"):
        ph = np.where(z != 0, np.arctan(y / np.where(z != 0, z, 1.0)), np.sign(y) * np.pi / 2)
    return th, ph


FOOTPRINTS = ("ewa", "ewa_snug", "ut", "ut_snug")


def footprint_bounds(scene, cam, method, **opts):
    """Projected-footprint association boxes in BEAP angles, FP64 -- the
    splatting associations the PBF is compared with (the EWA appendix and the
    association-method tables).  The camera-space Gaussian (mean mu_c, factor
    M = R_c R S, Sigma_c = M M^T) is projected by
      'ewa': the local affine approximation, angles of the mean and
             J Sigma_c J^T with J the Jacobian of (atan2(x, z), atan(y / z));
      'ut':  the unscented transform, sigma points mu_c and mu_c +- sqrt(3) m_k
             (columns of M) projected exactly, weights of alpha = 1, beta = 2,
             kappa = 0 (mean 1/6 per off-centre point; covariance 2 for the
             centre, 1/6 for the others), theta unwrapped around the centre's;
    and the box is centre +- lambda sqrt(largest eigenvalue) or, '_snug',
    centre +- lambda (sqrt(C_00), sqrt(C_11)), with lambda^2 the PBF's
    (conservative table value).  Returns dict(visible [N], tlo, thi, plo,
    phi) in radians; visible follows the FP32 cull and opacity decisions of
    the association reference."""
    a = assoc_fp32(scene, cam, **opts)
    o = opts_dict(**opts)
    n = scene.n
    Rc = np.asarray(cam["R"], np.float64)
    t = np.asarray(cam["t"], np.float64)
    mc = (Rc @ scene.mean.astype(np.float64)) + t[:, None]
    M = np.einsum("ab,nbc,cn->nac", Rc, _rotation(scene.quat.astype(np.float64)), scene.scale.astype(np.float64))
    L = np.array([lambda2_hat(float(sg), o["alpha_min"], o["lambda_mode"], o["lambda_fixed"]) for sg in
                  scene.opacity], np.float64)
    x, y, z = mc
    if method.startswith("ewa"):
        tc, pc = _beap(x, y, z)
        rxz, ryz = x * x + z * z, y * y + z * z
        with np.errstate(divide="ignore", invalid="ignore"):
            J = np.stack([np.stack([z / rxz, np.zeros(n), -x / rxz], -1),
                          np.stack([np.zeros(n), z / ryz, -y / ryz], -1)], 1)
        JM = J @ M
        Cv = JM @ np.transpose(JM, (0, 2, 1))
    else:
        t0, p0 = _beap(x, y, z)
        ts, ps = [], []
        for k in range(3):
            for sg in (np.sqrt(3.0), -np.sqrt(3.0)):
                pt = mc + sg * M[:, :, k].T
                tk, pk = _beap(*pt)
                ts.append(t0 + np.remainder(tk - t0 + np.pi, 2 * np.pi) - np.pi)
                ps.append(pk)
        ts, ps = np.array(ts), np.array(ps)
        tc, pc = ts.mean(0), ps.mean(0)
        dt, dp = np.vstack([t0 - tc, ts - tc]), np.vstack([p0 - pc, ps - pc])
        w = np.array([2.0] + [1 / 6] * 6)[:, None]
        Cv = np.stack([np.stack([(w * dt * dt).sum(0), (w * dt * dp).sum(0)], -1),
                       np.stack([(w * dt * dp).sum(0), (w * dp * dp).sum(0)], -1)], 1)
    c00, c01, c11 = Cv[:, 0, 0], Cv[:, 0, 1], Cv[:, 1, 1]
    if method.endswith("snug"):
        rt, rp = np.sqrt(L * c00), np.sqrt(L * c11)
    else:
        lam = 0.5 * (c00 + c11) + np.sqrt(0.25 * (c00 - c11) ** 2 + c01 ** 2)
        rt = rp = np.sqrt(L * lam)
    vis = (a["culled"] == 0) & (scene.opacity.astype(np.float32) > np.float32(o["alpha_min"]))
    vis &= np.isfinite(rt) & np.isfinite(rp) & np.isfinite(tc) & np.isfinite(pc)
    return dict(visible=vis, tlo=tc - rt, thi=tc + rt, plo=pc - rp, phi=pc + rp)


def angle_cells(edges, lo, hi, half, slack=0.0):
    """Half-tile cells [e[h], e[h+1]] met by the angle interval [lo, hi]
    (edges: tan(theta / 2) when `half`, else tan(phi)), with the interval
    grown by `slack` radians; an interval past -pi / pi wraps.  Returns
    (c0, c1), c0 > c1 when none."""
    lo, hi = lo - slack, hi + slack
    n = edges.size - 1
    pieces = []
    if half:
        if hi - lo >= 2 * np.pi:
            return 0, n - 1
        a = -np.inf if lo <= -np.pi else np.tan(lo / 2)
        b = np.inf if hi >= np.pi else np.tan(hi / 2)
        pieces.append((a, b))
        if lo < -np.pi:
            pieces.append((np.tan((lo + 2 * np.pi) / 2), np.inf))
        elif hi > np.pi:
            pieces.append((-np.inf, np.tan((hi - 2 * np.pi) / 2)))
    else:
        a = -np.inf if lo <= -np.pi / 2 else np.tan(lo)
        b = np.inf if hi >= np.pi / 2 else np.tan(hi)
        pieces.append((a, b))
    e = edges.astype(np.float64)
    c0, c1 = n, -1
    for a, b in pieces:
        hit = np.nonzero((e[1:] >= a) & (e[:-1] <= b))[0]
        if hit.size:
            c0, c1 = min(c0, hit[0]), max(c1, hit[-1])
    return c0, c1


def train_rows(sh_degree):
    return 11 + 3 * (sh_degree + 1) ** 2


def activate(raw):
    """Activated scale exp(log s) [3, n] and opacity sigmoid(logit) [n] of raw
    training rows (mean 3, log scale 3, quaternion 4, opacity logit 1, SH)."""
    raw = np.asarray(raw, np.float64)
    return np.exp(raw[3:6]), 1.0 / (1.0 + np.exp(-raw[10]))


def raw_gradients(raw, grads):
    """Gradients with respect to the raw rows from those with respect to the
    rendered parameters (mean, linear scale, quaternion, opacity, SH): the
    chain through s = exp(log s) and sigma = sigmoid(logit)."""
    scale, op = activate(raw)
    return np.concatenate([grads["mean"], grads["scale"] * scale, grads["quat"],
                           (grads["opacity"] * op * (1 - op))[None], grads["sh"]]).astype(np.float64)


def adam_step(raw, m, v, grads, step, lr, betas=(0.9, 0.999), eps=1e-15, accum=None, count=None):
    """One Adam step (Alg. "3DGEER Initialization and Training Framework") on
    raw rows, FP64: g = raw_gradients; m = b1 m + (1 - b1) g, v = b2 v +
    (1 - b2) g^2; raw -= lr_group m_hat / (sqrt(v_hat) + eps) with m_hat =
    m / (1 - b1^t), v_hat = v / (1 - b2^t); lr per group (mean, log scale,
    quaternion, opacity logit, SH).  The densification statistics add the
    mean gradient's norm and 1 where it is non-zero."""
    raw = np.asarray(raw, np.float64)
    g = raw_gradients(raw, grads)
    b1, b2 = betas
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    rate = np.concatenate([np.full(3, lr[0]), np.full(3, lr[1]), np.full(4, lr[2]), [lr[3]],
                           np.full(raw.shape[0] - 11, lr[4])])[:, None]
    new = raw - rate * (m / (1 - b1**step)) / (np.sqrt(v / (1 - b2**step)) + eps)
    out = dict(raw=new, m=m, v=v)
    out["scale"], out["opacity"] = activate(new)
    if accum is not None:
        gn = np.sqrt((g[0:3] ** 2).sum(0))
        out["accum"] = np.asarray(accum, np.float64) + gn
        out["count"] = np.asarray(count, np.float64) + (gn > 0)
    return out


def densify_kinds(raw, accum, count, grad_threshold, split_scale, min_opacity):
    """3DGS-style refinement decisions per Gaussian, in FP32 as the raw rows
    are held: 0 prune (opacity logit below logit(min_opacity)), 1 keep,
    2 clone, 3 split -- the last two when accum / count >= grad_threshold,
    split when the largest log scale exceeds log(split_scale)."""
    raw = np.asarray(raw, np.float32)
    prune = raw[10] < np.float32(math.log(min_opacity / (1 - min_opacity)))
    c = np.asarray(count, np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        avg = np.where(c > 0, np.asarray(accum, np.float32) / np.where(c > 0, c, np.float32(1)), np.float32(0))
    hot = (c > 0) & (avg >= np.float32(grad_threshold))
    big = raw[3:6].max(axis=0) > np.float32(math.log(split_scale))
    return np.where(prune, 0, np.where(hot, np.where(big, 3, 2), 1))


def densify(raw, m, v, accum, count, noise, grad_threshold, split_scale, min_opacity, split_shrink=1.6):
    """The refined training state, FP64, in input order: a kept Gaussian
    copied with its moments; a clone copied twice, the copy with zero
    moments; a split Gaussian replaced by two at mean + R S xi_c (xi_c =
    noise[3c:3c+3], R from the normalised quaternion) with log scale reduced
    by log(split_shrink) and zero moments; statistics reset."""
    raw = np.asarray(raw, np.float64)
    kinds = densify_kinds(raw, accum, count, grad_threshold, split_scale, min_opacity)
    cols, mm, vv = [], [], []
    Rall = _rotation(raw[6:10])
    s = np.exp(raw[3:6])
    for gi, k in enumerate(kinds):
        if k == 0:
            continue
        if k == 1 or k == 2:
            cols.append(raw[:, gi])
            mm.append(m[:, gi])
            vv.append(v[:, gi])
        if k == 2:
            cols.append(raw[:, gi])
            mm.append(np.zeros(raw.shape[0]))
            vv.append(np.zeros(raw.shape[0]))
        if k == 3:
            for c in range(2):
                x = raw[:, gi].copy()
                x[0:3] += Rall[gi] @ (s[:, gi] * np.asarray(noise, np.float64)[3 * c: 3 * c + 3, gi])
                x[3:6] -= math.log(split_shrink)
                cols.append(x)
                mm.append(np.zeros(raw.shape[0]))
                vv.append(np.zeros(raw.shape[0]))
    n = len(cols)
    R = raw.shape[0]
    out = dict(kinds=kinds, raw=np.array(cols).T.reshape(R, n), m=np.array(mm).T.reshape(R, n),
               v=np.array(vv).T.reshape(R, n), accum=np.zeros(n), count=np.zeros(n))
    out["scale"], out["opacity"] = activate(out["raw"])
    return out


def opts_dict(**kw):
    d = dict(DEFAULT_OPTS)
    d.update(kw)
    return d


__all__ = ["build", "assoc_fp32", "tile_list", "render", "branch_scores", "render_backward", "sh_basis", "pair", "edges",
           "lambda2_hat", "contrib_mask", "valid_mask", "kb_incidence", "reproject_positions", "reproject", "footprint_bounds", "angle_cells", "FOOTPRINTS",
           "train_rows", "activate", "raw_gradients", "adam_step", "densify_kinds", "densify", "pixel_dirs_camera", "pixel_dirs_world", "DEFAULT_OPTS"]


def tile_pairs_contribute(scene, cam, tiles, gids, nthreads: int = 0, **opts):
    """FP64: for each (tile, Gaussian) pair of one view, whether some ray of
    the 16x16 tile meets the contribution rule with the Gaussian."""
    tiles = np.ascontiguousarray(tiles, dtype=np.int32)
    gids = np.ascontiguousarray(gids, dtype=np.int64)
    out = np.zeros(tiles.size, np.uint8)
    ref = _SceneRef(scene)
    r = lib().orc_tile_pairs_contribute(C.byref(ref.c), C.byref(make_view(cam)), C.byref(make_opts(**opts)),
                                        tiles.size, _ptr(tiles), _ptr(gids), _ptr(out), int(nthreads))
    if r != 0:
        raise MemoryError("oracle allocation failed")
    return out.astype(bool)
