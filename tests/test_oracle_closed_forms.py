"""Pins of the FP64 oracle against closed forms, library routines and
quadrature -- nothing here re-types the oracle's own formulas.

* Eq. trans:cano / Thm. ray_splat: the ray opacity equals the line integral of
  the Gaussian density, checked by adaptive quadrature of the WORLD-space
  density (rotation built by scipy, not by the oracle's quaternion formula).
* Eq. mahdist_comp, isotropic case: kappa equals the textbook point-line
  distance squared over s^2.
* Eq. color: one- and two-Gaussian composites, transmittance bounds.
* SH basis (3DGS colour): orthonormality by exact product quadrature and
  agreement with scipy's complex spherical harmonics.
* BEAP (Sec. 3.3, App. E): pixel-centre directions round-trip to the
  (theta, phi) grid.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special
from scipy.spatial.transform import Rotation

import oracle
from paper_2505_24053_amd import synth


def one_gaussian(mu, s, q, sigma, rgb=(0.5, 0.5, 0.5)):
    sh = ((np.asarray(rgb, dtype=np.float64) - 0.5) / synth.SH_C0).reshape(3, 1)
    return synth.Scene(np.asarray(mu, np.float32).reshape(3, 1), np.asarray(s, np.float32).reshape(3, 1),
                       np.asarray(q, np.float32).reshape(4, 1), np.asarray([sigma], np.float32),
                       sh.astype(np.float32), 0)


def f64(scene, name):
    return getattr(scene, name).astype(np.float64)


def world_sigma(scene, g=0):
    q = f64(scene, "quat")[:, g]
    Rw = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scipy is scalar-last
    s = f64(scene, "scale")[:, g]
    return Rw @ np.diag(s**2) @ Rw.T


@pytest.mark.parametrize("seed", range(6))
def test_alpha_equals_world_line_integral(oracle_lib, seed):
    """sigma * int G_I(o_u + s d_u/|d_u|) ds over the canonical arc length
    equals sigma exp(-kappa/2); through the measure invariance of App. B this
    is the world-space line integral times |Sigma|^1/2 |Sigma^-1/2 d|."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform([-1, -1, 3], [1, 1, 6])
    s = np.exp(rng.uniform(np.log(0.05), np.log(0.4), 3))
    q = rng.standard_normal(4)
    sc = one_gaussian(mu, s, q, 0.8)
    cam = synth.camera_pinhole(64, 64, 60.0)
    mu64 = f64(sc, "mean")[:, 0]
    Sig = world_sigma(sc)
    Sinv = np.linalg.inv(Sig)
    for trial in range(4):
        d = mu64 + rng.normal(0, 0.6 * s.max(), 3)
        d /= np.linalg.norm(d)
        kappa, tstar, alpha, _ = oracle.pair(sc, cam, 0, d)
        norm = 1.0 / (math.sqrt(2 * math.pi) * math.sqrt(np.linalg.det(Sig)))
        dens = lambda t: norm * math.exp(-0.5 * (t * d - mu64) @ Sinv @ (t * d - mu64))
        tc = float(d @ Sinv @ mu64 / (d @ Sinv @ d))
        span = 12 * math.sqrt(np.linalg.eigvalsh(Sig).max())
        val, err = integrate.quad(dens, tc - span, tc + span, epsabs=1e-14, epsrel=1e-12, limit=200)
        expect = float(np.float32(0.8)) * val * math.sqrt(np.linalg.det(Sig)) * math.sqrt(d @ Sinv @ d)
        assert alpha == pytest.approx(expect, rel=1e-9, abs=1e-14)
        assert tstar == pytest.approx(tc, rel=1e-9)


def test_theorem_isotropic_integral_gauss_hermite():
    """Thm. ray_splat: int (1/sqrt(2 pi)) exp(-|u0 + t e|^2 / 2) dt = exp(-D^2/2)
    with D the point-line distance (the proof's 'D^2 = (u0^2+v0^2)/2' is a
    typo; the half is already in the exponent)."""
    x, w = np.polynomial.hermite.hermgauss(60)
    rng = np.random.default_rng(3)
    for _ in range(20):
        u0 = rng.normal(0, 2, 3)
        e = rng.normal(size=3)
        e /= np.linalg.norm(e)
        # substitute t = sqrt(2) y + t*, exp(-y^2) weight
        tstar = -u0 @ e
        perp = u0 + tstar * e
        D2 = perp @ perp
        vals = np.array([math.exp(-0.5 * np.sum((u0 + (math.sqrt(2) * y + tstar) * e) ** 2) + y * y) for y in x])
        integral = math.sqrt(2) * np.sum(w * vals) / math.sqrt(2 * math.pi)
        assert integral == pytest.approx(math.exp(-0.5 * D2), rel=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_isotropic_kappa_is_point_line_distance(oracle_lib, seed):
    rng = np.random.default_rng(100 + seed)
    mu = rng.uniform([-2, -2, 2], [2, 2, 8])
    s = float(np.exp(rng.uniform(np.log(0.02), np.log(0.5))))
    sc = one_gaussian(mu, [s, s, s], rng.standard_normal(4), 0.6)
    cam = synth.camera_pinhole(32, 32, 90.0)
    mu64 = f64(sc, "mean")[:, 0]
    s64 = float(f64(sc, "scale")[0, 0])
    for _ in range(5):
        d = rng.normal(size=3)
        d[2] = abs(d[2]) + 1
        d /= np.linalg.norm(d)
        kappa, tstar, alpha, lam2 = oracle.pair(sc, cam, 0, d)
        dist2 = np.sum(np.cross(mu64, d) ** 2)
        assert kappa == pytest.approx(dist2 / s64**2, rel=1e-10)
        assert tstar == pytest.approx(mu64 @ d, rel=1e-10)
        assert lam2 == pytest.approx(2 * math.log(float(np.float32(0.6)) * 255), rel=1e-12)


def test_kappa_special_cases(oracle_lib):
    sc = one_gaussian([0.3, -0.2, 4.0], [0.1, 0.3, 0.05], [0.9, 0.1, -0.3, 0.2], 0.7)
    cam = synth.camera_pinhole(32, 32, 60.0)
    mu = f64(sc, "mean")[:, 0]
    d = mu / np.linalg.norm(mu)
    kappa, tstar, alpha, _ = oracle.pair(sc, cam, 0, d)
    assert abs(kappa) < 1e-20
    assert alpha == pytest.approx(float(np.float32(0.7)), rel=1e-15)
    assert tstar == pytest.approx(np.linalg.norm(mu), rel=1e-12)
    # invariant to the length of d; t* scales inversely
    d2 = (d + np.array([0.01, -0.02, 0.0]))
    k1, t1, _, _ = oracle.pair(sc, cam, 0, d2)
    k2, t2, _, _ = oracle.pair(sc, cam, 0, 3.5 * d2)
    assert k2 == pytest.approx(k1, rel=1e-12)
    assert t2 == pytest.approx(t1 / 3.5, rel=1e-12)


def test_composite_one_and_two_gaussians(oracle_lib):
    """Eq. color with one and with two Gaussians on the optical axis."""
    mu = np.array([[0.0, 0.0], [0.0, 0.0], [3.0, 5.0]], np.float32)
    s = np.full((3, 2), 0.4, np.float32)
    q = np.array([[1, 1], [0, 0], [0, 0], [0, 0]], np.float32)
    sig = np.array([0.5, 0.7], np.float32)
    rgb = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    sh = ((rgb - 0.5) / synth.SH_C0).astype(np.float32)
    two = synth.Scene(mu, s, q, sig, sh, 0)
    cam = synth.camera_pinhole(16, 16, 30.0)
    pix = np.array([7 * 16 + 7, 8 * 16 + 8, 3 * 16 + 12])
    d = oracle.pixel_dirs_world(cam, pix)
    out2 = oracle.render(two, cam, pix=pix)
    out1 = oracle.render(two.subset([1]), cam, pix=pix)
    for t in range(pix.size):
        a = []
        for g in range(2):
            m = mu[:, g].astype(np.float64)
            s32 = float(np.float32(0.4))
            k = np.sum(np.cross(m, d[t]) ** 2) / s32**2
            a.append(float(sig[g]) * math.exp(-0.5 * k))
        c1 = rgb[:, 1] * a[1]
        assert out1["rgb"][t] == pytest.approx(c1, abs=1e-6)
        assert out1["trans"][t] == pytest.approx(1 - a[1], abs=1e-6)
        c2 = rgb[:, 0] * a[0] + rgb[:, 1] * a[1] * (1 - a[0])
        assert out2["rgb"][t] == pytest.approx(c2, abs=1e-6)
        assert out2["trans"][t] == pytest.approx((1 - a[0]) * (1 - a[1]), abs=1e-6)
        assert out2["ncomp"][t] == 2


def test_transmittance_bounds_and_termination(oracle_lib):
    sc, cams = synth.workload_small()
    cam = cams[0]
    r = oracle.render(sc, cam)
    T = r["trans"]
    assert np.all(T <= 1.0) and np.all(T >= 1e-4 * (1 - 1e-12))
    empty = r["ncomp"] == 0
    assert np.all(T[empty] == 1.0) and np.all(r["rgb"][empty] == 0)
    # without early termination, transmittance only falls further
    r0 = oracle.render(sc, cam, t_min=0.0)
    assert np.all(r0["trans"] <= T + 1e-15)
    assert np.all(r0["ncomp"] >= r["ncomp"])


def real_sh_scipy(deg, dirs):
    x, y, z = dirs.T
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    cols = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            if m == 0:
                cols.append(special.sph_harm_y(l, 0, theta, phi).real)
            elif m > 0:
                cols.append(math.sqrt(2) * special.sph_harm_y(l, m, theta, phi).real)
            else:
                cols.append(math.sqrt(2) * special.sph_harm_y(l, -m, theta, phi).imag)
    return np.stack(cols, -1)


def test_sh_matches_scipy_and_is_orthonormal(oracle_lib):
    rng = np.random.default_rng(5)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y, _ = oracle.sh_basis(3, d)
    np.testing.assert_allclose(Y, real_sh_scipy(3, d), atol=1e-12)
    # 3DGS's printed degree-0/1 constants follow from this basis
    assert Y[0, 0] == pytest.approx(0.28209479177387814)
    # exact product quadrature: Gauss-Legendre in z (20) x uniform phi (40)
    zl, wl = np.polynomial.legendre.leggauss(20)
    ph = np.arange(40) * 2 * np.pi / 40
    Z, P = np.meshgrid(zl, ph, indexing="ij")
    r = np.sqrt(1 - Z**2)
    dirs = np.stack([r * np.cos(P), r * np.sin(P), Z], -1).reshape(-1, 3)
    wts = (wl[:, None] * np.full(40, 2 * np.pi / 40)[None, :]).ravel()
    Yq, _ = oracle.sh_basis(3, dirs)
    G = (Yq * wts[:, None]).T @ Yq
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_gradient_matches_finite_differences(oracle_lib):
    rng = np.random.default_rng(6)
    d = rng.normal(size=(20, 3))
    _, dY = oracle.sh_basis(3, d)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        Yp, _ = oracle.sh_basis(3, d + e)
        Ym, _ = oracle.sh_basis(3, d - e)
        np.testing.assert_allclose(dY[:, :, a], (Yp - Ym) / (2 * h), rtol=1e-6, atol=1e-6)


def test_beap_directions_round_trip():
    for cam in (synth.camera_pinhole(40, 30, 60.0), synth.camera_equidistant(48, 48, 180.0),
                synth.camera_kb(64, 48, 200.0, seed=2)):
        w, h = cam["width"], cam["height"]
        pix = np.arange(w * h)
        d = oracle.pixel_dirs_camera(cam, pix)
        th = np.arctan2(d[:, 0], d[:, 2])
        ph = np.arctan(d[:, 1] / d[:, 2])
        px, py = pix % w, pix // w
        np.testing.assert_allclose(th, -cam["fov_x"] / 2 + (px + 0.5) * cam["fov_x"] / w, atol=1e-12)
        np.testing.assert_allclose(ph, -cam["fov_y"] / 2 + (py + 0.5) * cam["fov_y"] / h, atol=1e-12)
        np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)


def test_valid_mask_shapes():
    cam = synth.camera_pinhole(64, 48, 60.0)
    assert oracle.valid_mask(cam).all()
    kb = synth.camera_kb(128, 96, 190.0, seed=0)
    m = oracle.valid_mask(kb)
    assert m.all()  # BEAP box and sensor have the same angular extent
    # a BEAP grid wider than the sensor's field of view: outer columns invalid
    wide = dict(kb, fov_x=kb["fov_x"] * 1.2, fov_y=kb["fov_y"] * 1.2)
    m = oracle.valid_mask(wide)
    assert m[48, 64] and not m[48, 0] and not m[48, -1]
    assert 0.5 < m.mean() < 1.0


def _concat(*scenes):
    return synth.Scene(*(np.concatenate([getattr(s, k) for s in scenes], axis=-1)
                         for k in ("mean", "scale", "quat", "opacity", "sh")), 0)


def test_threshold_flags_only_before_latest_termination(oracle_lib):
    """A Gaussian whose kappa sits exactly on lambda^2 for the centre ray is a
    threshold-ambiguous pair.  Behind four opaque Gaussians that end the ray
    (T falls 0.05^4 < T_min) it cannot change the result and is not flagged;
    in front of them it is flagged, with a bound of 2 sigma max(c).  The
    colours are the closed-form composites of the opaque ones."""
    cam = synth.camera_pinhole(1, 1, 10.0)  # one ray along +z
    q = [1.0, 0.0, 0.0, 0.0]
    wall = [one_gaussian([0, 0, z], [0.1] * 3, q, 0.95, rgb=(0.2, 0.4, 0.6)) for z in (2.0, 3.0, 4.0, 5.0)]
    sig, s = 0.5, 0.3
    lam2 = 2 * math.log(float(np.float32(sig)) / (1 / 255))
    b = float(np.float32(s)) * math.sqrt(lam2)

    def edge(z):
        return one_gaussian([b, 0, z], [s] * 3, q, sig, rgb=(0.9, 0.1, 0.1))

    kappa, tstar, _, lam2_o = oracle.pair(edge(10.0), cam, 0, [0.0, 0.0, 1.0])
    assert kappa == pytest.approx(lam2, rel=1e-6) and lam2_o == pytest.approx(lam2, rel=1e-12) and tstar > 0
    a = 0.95
    c_wall = 0.2 * (a + a * (1 - a) + a * (1 - a) ** 2)  # three composited, the fourth ends the ray
    behind = oracle.render(_concat(*wall, edge(10.0)), cam)
    assert not behind["amb"][0]
    assert behind["ncomp"][0] == 3
    assert behind["rgb"][0, 0] == pytest.approx(c_wall, abs=1e-6)
    front = oracle.render(_concat(edge(1.0), *wall), cam)
    assert front["amb"][0]
    # its two branches: the edge Gaussian left out (the wall alone) or in,
    # with alpha = alpha_min in front of the wall
    n = int(front["branch_count"][0])
    red = sorted(front["branch_leaves"][0, :n, 0])
    ae = float(np.float32(sig)) * math.exp(-0.5 * kappa)
    assert n == 2
    assert red[0] == pytest.approx(c_wall, abs=1e-6)
    assert red[1] == pytest.approx(0.9 * ae + (1 - ae) * c_wall, abs=1e-6)
    # with no termination the pair behind is reachable again, hence flagged
    no_stop = oracle.render(_concat(*wall, edge(10.0)), cam, t_min=0.0)
    assert no_stop["amb"][0]


def test_termination_branches(oracle_lib):
    """Two clamped Gaussians (alpha = alpha_max = 0.99) on the ray take the
    transmittance to (1 - 0.99)^2 = 1e-4 = T_min: whether the second one
    blends is within FP32 error, so both outcomes are branches: stop before
    it (C = 0.99 c1) or blend it (C = 0.99 c1 + 0.99 * 0.01 c2)."""
    cam = synth.camera_pinhole(1, 1, 10.0)
    q = [1.0, 0.0, 0.0, 0.0]
    g1 = one_gaussian([0, 0, 2.0], [0.1] * 3, q, 0.999, rgb=(0.3, 0.0, 0.0))
    g2 = one_gaussian([0, 0, 3.0], [0.1] * 3, q, 0.999, rgb=(0.8, 0.0, 0.0))
    out = oracle.render(_concat(g1, g2), cam)
    assert out["amb"][0]
    n = int(out["branch_count"][0])
    leaves = out["branch_leaves"][0, :n]
    red = sorted(leaves[:, 0])
    assert n == 2
    assert red[0] == pytest.approx(0.99 * 0.3, abs=1e-6)
    assert red[1] == pytest.approx(0.99 * 0.3 + 0.99 * 0.01 * 0.8, abs=1e-6)
    assert sorted(leaves[:, 4]) == pytest.approx([0.01 * 0.01, 0.01], rel=1e-9)
    # well away from T_min (a third of the opacity) there is one outcome
    g3 = one_gaussian([0, 0, 3.0], [0.1] * 3, q, 0.3, rgb=(0.8, 0.0, 0.0))
    one = oracle.render(_concat(g1, g3), cam)
    assert not one["amb"][0] and one["branch_idx"].size == 0
