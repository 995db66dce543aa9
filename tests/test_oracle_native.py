"""Pins of the oracle's native-space resampling (App. E inverse
interpolation): the grid positions it finds for native pixel centres are
checked by projecting them back through the paper's printed camera models,
and the interpolation by images whose bilinear interpolation is known."""
import math

import numpy as np
import pytest

import oracle
from paper_2505_24053_amd import synth


def beap_angles(cam, gx, gy):
    th = -cam["fov_x"] / 2 + (gx + 0.5) * cam["fov_x"] / cam["width"]
    ph = -cam["fov_y"] / 2 + (gy + 0.5) * cam["fov_y"] / cam["height"]
    return th, ph


def project_printed(cam, th, ph):
    """App. E forward models, as printed (rays in front of the camera):
    pinhole x_p = f_x tan(theta) + c_x; KB r = sqrt(tan^2 theta + tan^2 phi),
    incidence atan(r), distorted angle phi_d, x_p = f_x phi_d / r tan(theta)
    + c_x (likewise y_p)."""
    tt, tp = np.tan(th), np.tan(ph)
    if cam["model"] == "pinhole":
        return cam["fx"] * tt + cam["cx"], cam["fy"] * tp + cam["cy"]
    k = cam["k"]
    r = np.sqrt(tt**2 + tp**2)
    a = np.arctan(r)
    ad = a * (1 + k[0] * a**2 + k[1] * a**4 + k[2] * a**6 + k[3] * a**8)
    s = np.where(r > 0, ad / np.where(r > 0, r, 1.0), 1.0)
    return cam["fx"] * s * tt + cam["cx"], cam["fy"] * s * tp + cam["cy"]


CAMS = {
    "pinhole60": synth.camera_pinhole(96, 72, 60.0),
    "equidistant180": synth.camera_equidistant(96, 96, 180.0),
    "kb190": synth.camera_kb(128, 96, 190.0, seed=0),
    "kb200": synth.camera_kb(120, 68, 200.0, seed=4),
}


@pytest.mark.parametrize("name", list(CAMS))
def test_positions_project_back_to_pixel_centres(name):
    cam = CAMS[name]
    gx, gy, ok = oracle.reproject_positions(cam)
    # the BEAP box of the KB cameras (equal angular pitch) covers the sensor's
    # central band only: their strong distortion maps the sensor's vertical
    # extent beyond the box's vertical FoV
    assert ok.mean() > 0.2
    th, ph = beap_angles(cam, gx, gy)
    front = ok & (np.abs(th) < math.pi / 2 - 1e-3)
    assert front.sum() > 100
    u, v = project_printed(cam, th[front], ph[front])
    jj, ii = np.nonzero(front)
    np.testing.assert_allclose(u, ii + 0.5, atol=1e-9)
    np.testing.assert_allclose(v, jj + 0.5, atol=1e-9)


def test_kb_incidence_inverts_the_distortion():
    k = synth.kb_coeffs(3, 190.0)
    th = np.linspace(0.0, math.radians(95.0), 1001)
    td = th * (1 + k[0] * th**2 + k[1] * th**4 + k[2] * th**6 + k[3] * th**8)
    np.testing.assert_allclose(oracle.kb_incidence(td, k), th, atol=1e-14)
    # past the end of the increasing branch no ray lands
    kneg = [-0.2, 0.0, 0.0, 0.0]  # theta - 0.2 theta^3 peaks at theta = sqrt(5/3)
    peak = math.sqrt(5 / 3) * (1 - 0.2 * 5 / 3)
    assert np.isnan(oracle.kb_incidence([peak * 1.001], kneg))[0]
    assert np.isfinite(oracle.kb_incidence([peak * 0.999], kneg))[0]


@pytest.mark.parametrize("name", list(CAMS))
def test_bilinear_reproduces_affine_images(name):
    """Bilinear interpolation is exact on images affine in the grid position,
    so at a reached pixel the value is a + b x + c y of its position (after
    clamping into the grid)."""
    cam = CAMS[name]
    w, h = cam["width"], cam["height"]
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    coef = [(0.3, 0.01, -0.02), (1.0, 0.0, 0.0), (-0.5, 0.003, 0.007)]
    img = np.stack([a + b * xx + c * yy for a, b, c in coef])
    nat, ok = oracle.reproject(cam, img)
    gx, gy, ok2 = oracle.reproject_positions(cam)
    assert (ok == ok2).all()
    x, y = np.clip(gx, 0, w - 1), np.clip(gy, 0, h - 1)
    for ch, (a, b, c) in enumerate(coef):
        np.testing.assert_allclose(nat[ch][ok], (a + b * x + c * y)[ok], atol=1e-12)
        assert (nat[ch][~ok] == 0).all()


def test_native_size_and_unreached_pixels():
    """A native sensor larger than the BEAP box: pixels past the grid's
    angular extent are unreached; a sensor with the grid's size and matching
    extent is reached everywhere (the synthetic cameras map the half FoV to
    the sensor edge)."""
    cam = CAMS["kb190"]
    _, _, ok = oracle.reproject_positions(cam, native_size=(cam["width"] + 40, cam["height"] + 40))
    assert not ok.all() and ok.any()
    pin = CAMS["pinhole60"]
    _, _, okp = oracle.reproject_positions(pin)
    assert okp.all()


NATIVE = [synth.camera_pinhole_native(40, 32, 70.0), synth.camera_pinhole_native(37, 29, 100.0, principal=(0.3, 0.6),
                                                                                  aspect=1.1)]


@pytest.mark.parametrize("cam", NATIVE, ids=["centred", "offset_principal"])
def test_native_grid_rays_hit_their_pixel_centres(cam):
    """A native pinhole grid's rays project, through the pinhole model of
    App. E, onto their own pixel centres."""
    w, h = cam["width"], cam["height"]
    d = oracle.pixel_dirs_camera(cam, np.arange(w * h))
    u = cam["fx"] * d[:, 0] / d[:, 2] + cam["cx"]
    v = cam["fy"] * d[:, 1] / d[:, 2] + cam["cy"]
    np.testing.assert_allclose(u, np.arange(w * h) % w + 0.5, atol=1e-9)
    np.testing.assert_allclose(v, np.arange(w * h) // w + 0.5, atol=1e-9)
    assert oracle.valid_mask(cam).all()


@pytest.mark.parametrize("cam", NATIVE, ids=["centred", "offset_principal"])
def test_native_grid_edges_bracket_pixel_rays(cam):
    """Each half-tile's edges (mirrored tan(theta/2) columns, tan(phi) rows)
    bracket the BEAP angles of its pixels' rays."""
    ex, ey = oracle.edges(cam)
    w, h = cam["width"], cam["height"]
    d = oracle.pixel_dirs_camera(cam, np.arange(w * h))
    th = np.arctan2(d[:, 0], d[:, 2])
    ph = np.arctan2(d[:, 1], d[:, 2])
    px, py = np.arange(w * h) % w, np.arange(w * h) // w
    t2 = np.tan(th / 2)
    assert np.all(ex[px // 8] < t2) and np.all(t2 < ex[px // 8 + 1])
    tp = np.tan(ph)
    assert np.all(ey[py // 8] < tp) and np.all(tp < ey[py // 8 + 1])


@pytest.mark.parametrize("seed", range(3))
def test_native_grid_association_superset(oracle_lib, seed):
    """Every contributing (ray, Gaussian) pair of a native pinhole grid lies
    in the Gaussian's half-tile rectangle (brute force)."""
    from helpers import adversarial_scene
    from test_oracle_association import check_superset

    rng = np.random.default_rng(70 + seed)
    R, c = synth.random_pose(rng, half=1.0)
    cam = synth.camera_pinhole_native(40, 32, 90.0, R, c, principal=(0.4, 0.55))
    assert check_superset(adversarial_scene(seed + 20), cam) > 0
