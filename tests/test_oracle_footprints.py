"""Pins of the oracle's projected-footprint associations (EWA local affine
approximation and unscented transform in BEAP angles), the baselines the PBF
is compared with."""
import math

import numpy as np
import pytest

import oracle
from paper_2505_24053_amd import synth


def one(mu, s, q=(1.0, 0.0, 0.0, 0.0), sigma=0.8):
    return synth.Scene(np.asarray(mu, np.float32).reshape(3, 1), np.asarray(s, np.float32).reshape(3, 1),
                       np.asarray(q, np.float32).reshape(4, 1), np.asarray([sigma], np.float32),
                       np.zeros((3, 1), np.float32), 0)


@pytest.mark.parametrize("method", oracle.FOOTPRINTS)
def test_small_far_isotropic_matches_tangent_angle(method):
    """A small isotropic Gaussian on the optical axis: every footprint's
    half-width tends to the exact tangent half-angle asin(lambda s / z) of the
    PBF closed form, to first order in s / z."""
    cam = synth.camera_equidistant(64, 64, 180.0)
    z, s = 5.0, 0.002
    b = oracle.footprint_bounds(one([0, 0, z], [s] * 3), cam, method)
    lam = math.sqrt(oracle.lambda2_hat(0.8))
    exact = math.asin(lam * s / z)
    assert b["visible"][0]
    for lo, hi in ((b["tlo"][0], b["thi"][0]), (b["plo"][0], b["phi"][0])):
        assert abs(0.5 * (lo + hi)) < 1e-12
        assert 0.5 * (hi - lo) == pytest.approx(exact, rel=1e-5)


def test_ewa_jacobian_is_the_angle_maps_derivative():
    """EWA's covariance J Sigma J^T with the analytic Jacobian equals the one
    from central differences of the BEAP angle map at the mean."""
    rng = np.random.default_rng(3)
    cam = synth.camera_equidistant(64, 64, 180.0)
    for _ in range(20):
        mu = rng.normal(0, 2, 3)
        mu[2] = abs(mu[2]) + 0.5
        s = np.exp(rng.uniform(-4, -1, 3))
        q = rng.normal(size=4)
        sc = one(mu, s, q)
        b = oracle.footprint_bounds(sc, cam, "ewa_snug")
        R = oracle._rotation(sc.quat.astype(np.float64))[0]
        M = R * sc.scale.astype(np.float64)[:, 0]
        m = sc.mean.astype(np.float64)[:, 0]
        J = np.zeros((2, 3))
        for a in range(3):
            e = np.zeros(3)
            e[a] = 1e-6
            tp = np.array(oracle._beap(*(m + e)))
            tm = np.array(oracle._beap(*(m - e)))
            J[:, a] = (tp - tm) / 2e-6
        C = J @ M @ M.T @ J.T
        lam2 = oracle.lambda2_hat(0.8)
        assert 0.5 * (b["thi"][0] - b["tlo"][0]) == pytest.approx(math.sqrt(lam2 * C[0, 0]), rel=1e-6)
        assert 0.5 * (b["phi"][0] - b["plo"][0]) == pytest.approx(math.sqrt(lam2 * C[1, 1]), rel=1e-6)


def test_ut_is_exact_for_linear_maps_and_square_box_covers_snug():
    """For a Gaussian far from the camera the projection is nearly linear over
    it, so the unscented covariance agrees with EWA's; the square box (largest
    eigenvalue) always contains the snug one."""
    sc = synth.scene_box(300, seed=4, half=3.0, smax=0.05)
    sc.mean[2] += 40.0
    cam = synth.camera_pinhole(64, 64, 30.0)
    e, u = oracle.footprint_bounds(sc, cam, "ewa_snug"), oracle.footprint_bounds(sc, cam, "ut_snug")
    v = e["visible"] & u["visible"]
    assert v.sum() > 250
    np.testing.assert_allclose(u["thi"][v] - u["tlo"][v], e["thi"][v] - e["tlo"][v], rtol=2e-3)
    np.testing.assert_allclose(u["phi"][v] - u["plo"][v], e["phi"][v] - e["plo"][v], rtol=2e-3)
    sq = oracle.footprint_bounds(sc, cam, "ewa")
    assert np.all(sq["thi"][v] - sq["tlo"][v] >= e["thi"][v] - e["tlo"][v] - 1e-12)


def test_footprints_miss_contributions_the_pbf_keeps():
    """Near, large Gaussians seen off-axis through a 180-degree fisheye: the
    footprint boxes leave out (ray, Gaussian) pairs that contribute, which the
    PBF rectangle never does."""
    from test_oracle_association import check_superset

    rng = np.random.default_rng(8)
    n = 40
    d = rng.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    d[2] = np.abs(d[2]) * 0.5
    mu = d * rng.uniform(0.8, 2.0, n)
    sc = synth.Scene(mu.astype(np.float32), rng.uniform(0.15, 0.3, (3, n)).astype(np.float32),
                     rng.normal(size=(4, n)).astype(np.float32), rng.uniform(0.5, 0.9, n).astype(np.float32),
                     np.zeros((3, n), np.float32), 0)
    cam = synth.camera_equidistant(48, 48, 180.0)
    assert check_superset(sc, cam) > 0  # the PBF misses nothing
    mask = oracle.contrib_mask(sc, cam)
    ex, ey = oracle.edges(cam)
    pix = np.arange(48 * 48)
    hx, hy = (pix % 48) // 8, (pix // 48) // 8
    missed = 0
    for method in ("ewa", "ut"):
        b = oracle.footprint_bounds(sc, cam, method)
        for g in range(n):
            rays = np.nonzero(mask[:, g])[0]
            if rays.size == 0:
                continue
            if not b["visible"][g]:
                missed += rays.size
                continue
            x0, x1 = oracle.angle_cells(ex, b["tlo"][g], b["thi"][g], True)
            y0, y1 = oracle.angle_cells(ey, b["plo"][g], b["phi"][g], False)
            inside = (hx[rays] >= x0) & (hx[rays] <= x1) & (hy[rays] >= y0) & (hy[rays] <= y1)
            missed += int((~inside).sum())
    assert missed > 0
