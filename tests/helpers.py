"""Shared inputs and comparisons of the test suite."""
import numpy as np

import oracle

from paper_2505_24053_amd import synth


def adversarial_scene(seed, n=48):
    """Camera at the origin looking down +z; Gaussians placed where the
    association is hard."""
    rng = np.random.default_rng(seed)
    mu = np.zeros((3, n))
    s = np.exp(rng.uniform(np.log(0.01), np.log(0.6), (3, n)))
    kinds = rng.integers(0, 8, n)
    for g in range(n):
        k = kinds[g]
        if k == 0:  # anywhere around the camera, including behind
            d = rng.normal(size=3)
            mu[:, g] = d / np.linalg.norm(d) * rng.uniform(0.4, 5.0)
        elif k == 1:  # straddling the z = 0 plane
            mu[:, g] = [rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-0.3, 0.3)]
        elif k == 2:  # near the camera y axis (theta pencil)
            mu[:, g] = [rng.normal(0, 0.2), rng.uniform(-3, 3), rng.normal(0, 0.2)]
        elif k == 3:  # near the camera x axis (phi pencil)
            mu[:, g] = [rng.uniform(-3, 3), rng.normal(0, 0.2), rng.normal(0, 0.2)]
        elif k == 4:  # disk: one tiny scale
            mu[:, g] = [rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.5, 4)]
            s[rng.integers(0, 3), g] = 1e-6 * s[:, g].max()
        elif k == 5:  # needle: two tiny scales
            mu[:, g] = [rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(-1, 4)]
            a = rng.permutation(3)[:2]
            s[a, g] = 1e-6 * s[:, g].max()
        elif k == 6:  # camera just outside 3 sigma
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            s[:, g] = rng.uniform(0.3, 0.8)
            mu[:, g] = d * s[0, g] * rng.uniform(3.0, 3.6)
        else:  # beside the camera, large
            mu[:, g] = [rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(-2, 2)]
            s[:, g] = rng.uniform(0.2, 1.0, 3)
    q = rng.standard_normal((4, n))
    sig = rng.uniform(0.02, 0.99, n)
    sh = rng.normal(0, 0.3, (3, n))
    return synth.Scene(mu.astype(np.float32), s.astype(np.float32), q.astype(np.float32),
                       sig.astype(np.float32), sh.astype(np.float32), 0)


RGB_TOL = 2e-4  # RGB max-abs gate, FP32 GPU vs FP64 oracle


FLAGGED_MAX = 0.05  # largest share of rays with an FP32-ambiguous decision


def compare_render(got, ref, pix=None, rgb_tol=RGB_TOL, flagged_max=FLAGGED_MAX):
    """GPU rays against the FP64 oracle (Eq. color).  A ray whose decisions
    all lie outside the FP32 error band must match the FP64 result: RGB and T
    within rgb_tol, depth within 1e-3 relative.  A flagged ray must match one
    of its decision branches (each flagged contribution in or out, each
    ambiguous termination taken or not) within the same gates."""
    sel = slice(None) if pix is None else pix
    g_rgb, g_d, g_t = got["rgb"][sel], got["depth"][sel], got["trans"][sel]
    amb = ref["amb"]
    ok = ~amb
    err = np.abs(g_rgb - ref["rgb"]).max(axis=1)
    assert err[ok].max(initial=0) <= rgb_tol, "max |rgb| err %g at %s" % (err[ok].max(), np.argmax(np.where(ok, err, 0)))
    terr = np.abs(g_t - ref["trans"])
    assert terr[ok].max(initial=0) <= rgb_tol, "max |T| err %g" % terr[ok].max()
    derr = np.abs(g_d - ref["depth"]) / (1.0 + np.abs(ref["depth"]))
    assert derr[ok].max(initial=0) <= 1e-3, "max depth rel err %g" % derr[ok].max()
    score = oracle.branch_scores(g_rgb, g_d, g_t, ref, rgb_tol)
    assert score.max(initial=0) <= 1.0, "flagged ray matches no branch: score %g at %s (%d branches)" % (
        score.max(), ref["branch_idx"][np.argmax(score)], ref["branch_count"][np.argmax(score)])
    assert amb.mean() <= flagged_max, "flagged share %.4f" % amb.mean()
    print("rays %d, flagged %d (%.3f%%), each within the gates of one branch (max %d branches); "
          "max err unflagged %.3g" % (amb.size, amb.sum(), 100 * amb.mean(),
                                      int(ref["branch_count"].max(initial=1)), err[ok].max(initial=0)))
    return float(err[ok].max(initial=0)), int(amb.sum())


def heavy_pixel_mask(ranges, cams):
    """Per ray (views concatenated) whether its 16x16 tile is heavy under the
    renderer's rule: list longer than 3x the mean over the tiles of its own
    view, plus 64.  Heavy tiles composite four entries per step, which rounds
    differently from the one-entry steps of ordinary tiles."""
    import numpy as np
    cnt = np.diff(np.asarray(ranges, dtype=np.int64))
    masks, base = [], 0
    for cam in cams:
        w, h = cam["width"], cam["height"]
        tx, ty = (w + 15) // 16, (h + 15) // 16
        c = cnt[base:base + tx * ty]
        heavy = (c > 3 * int(c.sum()) // c.size + 64).reshape(ty, tx)
        ys, xs = np.mgrid[0:h, 0:w]
        masks.append(heavy[ys // 16, xs // 16].ravel())
        base += tx * ty
    return np.concatenate(masks)
