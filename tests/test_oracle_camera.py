"""Pins of the valid-ray mask (App. E: BEAP rays projected through the
pinhole and Kannala-Brandt models onto the native sensor).

The oracle's ``valid_mask`` and the library's ``geer_valid_mask`` evaluate the
general projection (incidence angle atan2(|xy|, z), distortion polynomial,
azimuth).  Along three lines of an odd-sized BEAP grid the projection has a
closed form that involves none of that machinery, written out here:

* the centre row (phi = 0): the ray is (sin t, 0, cos t), its incidence is
  |t| and it lands on the horizontal line through the principal point;
* the centre column (theta = 0): the ray is (0, sin p, cos p), incidence |p|,
  vertical line;
* the diagonal theta = phi of a square grid: the ray is proportional to
  (tan t, tan t, 1), incidence atan(sqrt 2 |tan t|), azimuth 45 degrees.

The distortion is written as theta + k1 theta^3 + ... + k4 theta^9 with four
different coefficients, so a wrong power, a swapped coefficient or a missing
term moves the mask's edge on these lines.
"""
import math

import numpy as np
import pytest

import oracle


def grid(n, fov):
    return np.array([-fov / 2 + (i + 0.5) * fov / n for i in range(n)])


def cam(model, n, fov_deg, f, k=(0.0, 0.0, 0.0, 0.0), cx=None, cy=None):
    fov = math.radians(fov_deg)
    return dict(model=model, width=n, height=n, fx=f, fy=f, cx=n / 2 if cx is None else cx,
                cy=n / 2 if cy is None else cy, k=list(k), fov_x=fov, fov_y=fov, R=np.eye(3), t=np.zeros(3))


def distort(a, k):
    return a + k[0] * a**3 + k[1] * a**5 + k[2] * a**7 + k[3] * a**9


def on_sensor(u, v, n):
    return (u >= 0) & (u < n) & (v >= 0) & (v < n)


def masks(c):
    from paper_2505_24053_amd import _lib

    out = [oracle.valid_mask(c)]
    try:
        out.append(_lib.valid_mask(c))
    except OSError:  # the HIP runtime libraries are not loadable here
        pass
    return out


CASES = [
    ("equidistant", 65, 170.0, 31.3, (0.0, 0.0, 0.0, 0.0)),
    ("kb", 65, 170.0, 33.7, (0.031, -0.012, 0.0047, -0.0009)),
    ("kb", 81, 176.0, 41.9, (-0.04, 0.02, -0.006, 0.0011)),
    ("pinhole", 65, 150.0, 27.3, (0.0, 0.0, 0.0, 0.0)),
]


@pytest.mark.parametrize("model,n,fov,f,k", CASES)
def test_valid_mask_closed_form_lines(model, n, fov, f, k):
    c = cam(model, n, fov, f, k)
    t = grid(n, math.radians(fov))
    mid = n // 2
    assert abs(t[mid]) < 1e-12
    cx = cy = n / 2
    if model == "pinhole":
        row_u = cx + f * np.tan(t)          # theta lines: x / z = tan(theta)
        col_v = cy + f * np.tan(t)
        diag = f * np.tan(t)                # (tan t, tan t, 1): both offsets f tan t
        front = np.abs(t) < math.pi / 2
    else:
        row_u = cx + f * np.sign(t) * distort(np.abs(t), k)
        col_v = cy + f * np.sign(t) * distort(np.abs(t), k)
        psi = np.arctan(math.sqrt(2) * np.abs(np.tan(t)))
        diag = f * np.sign(t) * distort(psi, k) / math.sqrt(2)
        front = np.ones(n, bool)
    exp_row = front & on_sensor(row_u, np.full(n, cy), n)
    exp_col = front & on_sensor(np.full(n, cx), col_v, n)
    exp_diag = front & on_sensor(cx + diag, cy + diag, n)
    # the lines cross the sensor edge inside the grid, away from pixel centres
    for e in (exp_row, exp_col, exp_diag):
        assert e.any() and not e.all()
    for m in masks(c):
        np.testing.assert_array_equal(m[mid, :], exp_row)
        np.testing.assert_array_equal(m[:, mid], exp_col)
        np.testing.assert_array_equal(np.diagonal(m), exp_diag)


def test_valid_mask_beyond_90_degrees():
    """Rays past 90 degrees (z < 0) are invisible to a pinhole and visible to
    a fisheye whose distortion keeps them on the sensor."""
    n = 65
    t = grid(n, math.radians(250.0))
    pin = dict(cam("pinhole", n, 250.0, 10.0), height=33, cy=16.5, fov_y=math.radians(120.0))
    fish = dict(cam("equidistant", n, 250.0, (n / 2) / math.radians(130.0)), height=33, cy=16.5,
                fov_y=math.radians(120.0))
    back = np.abs(t) > math.pi / 2
    assert back.any()
    for m in masks(pin):
        assert not m[16, back].any()
    for m in masks(fish):
        assert m[16, :].all()  # |theta| <= 125 deg lands within the 130-deg radius
