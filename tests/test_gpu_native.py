"""Native camera-space output on the GPU against the oracle.

* geer_reproject (App. E inverse interpolation) on seeded images of every
  camera model: reached pixels bit for bit the same set, values within 1e-5
  of the FP64 bilinear interpolation (inputs in [0, 1]);
* end to end: a rendered BEAP frame resampled onto the native sensor,
  against the FP64 interpolation of the oracle's own rays at the four BEAP
  neighbours (on native pixels whose neighbours hold no FP32-ambiguous
  decision), RGB within the 2e-4 gate.
"""
import numpy as np
import pytest

import oracle
from paper_2505_24053_amd import _lib, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_24053_amd import renderer

    return renderer


CAMS = {
    "pinhole60": (synth.camera_pinhole(160, 120, 60.0), None),
    "equidistant180": (synth.camera_equidistant(200, 200, 180.0), None),
    "kb190": (synth.camera_kb(256, 192, 190.0, seed=0), None),
    "kb200_larger_sensor": (synth.camera_kb(240, 136, 200.0, seed=4), (300, 170)),
    "ragged": (synth.camera_kb(37, 23, 190.0, seed=2), (41, 29)),
}


@pytest.mark.parametrize("name", list(CAMS))
def test_reproject_matches_oracle(R, name):
    cam, size = CAMS[name]
    w, h = cam["width"], cam["height"]
    rng = np.random.default_rng(5)
    yy, xx = np.mgrid[0:h, 0:w]
    img = np.stack([rng.uniform(0, 1, (h, w)), 0.5 + 0.5 * np.sin(xx / 7.0) * np.cos(yy / 5.0),
                    rng.uniform(0, 1, (h, w)) ** 3, np.full((h, w), 0.25), (xx + yy) / (w + h)]).astype(np.float32)
    ref, ok = oracle.reproject(cam, img.astype(np.float64), native_size=size)
    for _ in range(2):  # the second call uses the cached map
        nat, valid = R.reproject(torch.as_tensor(img, device="cuda"), cam, native_size=size)
        torch.cuda.synchronize()
        got = nat.double().cpu().numpy()
        v = valid.cpu().numpy().astype(bool)
        np.testing.assert_array_equal(v, ok)
        assert np.abs(got - ref).max() <= 1e-5, np.abs(got - ref).max()
        assert (got[:, ~v] == 0).all()
    print("%s: %d of %d native pixels reached, max err %.2g" % (name, ok.sum(), ok.size, np.abs(got - ref).max()))


def test_reproject_rendered_frame_against_oracle_rays(R):
    scene = synth.scene_box(3000, seed=9, half=4.0)
    cam = synth.camera_kb(96, 72, 190.0, seed=1)
    sc = R.scene_from_numpy(scene)
    rgb, depth, trans, _ = R.render(sc, [cam])
    beap = torch.cat([rgb.view(3, -1), depth.view(1, -1), trans.view(1, -1)])
    nat, valid = R.reproject(beap, cam)
    torch.cuda.synchronize()
    gx, gy, ok = oracle.reproject_positions(cam)
    w, h = cam["width"], cam["height"]
    js, is_ = np.nonzero(ok)
    pick = np.random.default_rng(3).choice(js.size, min(600, js.size), replace=False)
    js, is_ = js[pick], is_[pick]
    x = np.clip(gx[js, is_], 0, w - 1)
    y = np.clip(gy[js, is_], 0, h - 1)
    x0, y0 = np.floor(x).astype(int), np.floor(y).astype(int)
    x1, y1 = np.minimum(x0 + 1, w - 1), np.minimum(y0 + 1, h - 1)
    corners = [(x0, y0), (x1, y0), (x0, y1), (x1, y1)]
    pix = np.unique(np.concatenate([cy * w + cx for cx, cy in corners]))
    ref = oracle.render(scene, cam, pix=pix)
    col = {int(p): k for k, p in enumerate(pix)}
    fx, fy = x - x0, y - y0
    wts = [(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy]
    exp = np.zeros((len(js), 5))
    clean = np.ones(len(js), bool)
    for (cx, cy), wt in zip(corners, wts):
        idx = np.array([col[int(p)] for p in cy * w + cx])
        vals = np.concatenate([ref["rgb"][idx], ref["depth"][idx, None], ref["trans"][idx, None]], axis=1)
        exp += wt[:, None] * vals
        clean &= ~ref["amb"][idx]
    got = nat.double().cpu().numpy()[:, js, is_].T
    assert valid.cpu().numpy()[js, is_].all()
    err = np.abs(got - exp)[clean]
    assert clean.mean() > 0.9
    assert err[:, :3].max() <= 2e-4 and err[:, 4].max() <= 2e-4, err.max(axis=0)
    assert (err[:, 3] / (1 + np.abs(exp[clean, 3]))).max() <= 1e-3
    print("end to end: %d native pixels, max rgb err %.2g" % (clean.sum(), err[:, :3].max()))


def test_reproject_rejects_bad_arguments(R):
    cam, _ = CAMS["pinhole60"]
    img = torch.zeros(3 * cam["width"] * cam["height"] + 1, device="cuda")
    with pytest.raises(ValueError):
        R.reproject(img, cam)
    with pytest.raises(_lib.GeerError):
        R.reproject(torch.zeros(3 * cam["width"] * cam["height"], device="cuda"), dict(cam, fx=0.0))


@pytest.mark.parametrize("kind", ["box", "adversarial", "large"])
def test_native_pinhole_grid_matches_oracle(R, kind):
    """Rendering straight onto a pinhole sensor's own pixels (only the edge
    and direction tables differ from a BEAP grid): association bit-exact
    against the FP32 reference, every ray against the FP64 oracle."""
    from helpers import adversarial_scene, compare_render
    from test_gpu_forward import check_association, gpu_render

    rng = np.random.default_rng(31)
    if kind == "box":
        scene = synth.scene_box(4000, seed=12, half=4.0)
        cam = synth.camera_pinhole_native(96, 72, 80.0, principal=(0.45, 0.55), aspect=1.05)
        pix = None
    elif kind == "adversarial":
        scene = adversarial_scene(21, n=64)
        Rm, c = synth.random_pose(rng, half=0.5)
        cam = synth.camera_pinhole_native(61, 45, 110.0, Rm, c)
        pix = None
    else:
        scene = synth.scene_box(100_000, seed=0)
        cam = synth.camera_pinhole_native(1280, 960, 90.0)
        pix = np.random.default_rng(4).choice(1280 * 960, 4096, replace=False)
    got, frame = gpu_render(R, scene, [cam])
    check_association(frame, scene, [cam])
    frame.release()
    ref = oracle.render(scene, cam, pix=pix)
    compare_render(got[0], ref, pix=pix)
