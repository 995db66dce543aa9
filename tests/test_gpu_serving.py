"""Render plans (captured graphs) and the continuous-batching server.

* a plan launch equals the eager render of the same cameras bit for bit, on
  repeated launches with new cameras of the same grid sizes;
* a batch that overflows the plan's association capacity is reported and
  renders background, and the plan recovers on the next launch;
* served results equal the same cameras rendered alone, bit for bit, for a
  Poisson mix of pinhole / equidistant / Kannala-Brandt requests of three
  resolutions, with batches of several views forming and batches of
  different slots in flight at once; one served request is also checked
  against the FP64 oracle on sampled rays;
* at the full serving size (1M Gaussians SH3; 640x480, 1024x1024 and
  1920x1080 requests) served results equal the alone renders and match the
  oracle on sampled rays.
"""
import numpy as np
import pytest

import oracle
from helpers import compare_render
from paper_2505_24053_amd import _lib, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_24053_amd import renderer

    if not __import__("os").path.exists(_lib.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return renderer


def small_cams(rng, kinds, half=3.0):
    cams = []
    for k in kinds:
        Rm, c = synth.random_pose(rng, half)
        if k == 0:
            cams.append(synth.camera_pinhole(80, 60, 60.0, Rm, c))
        elif k == 1:
            cams.append(synth.camera_equidistant(128, 128, 180.0, Rm, c))
        else:
            cams.append(synth.camera_kb(192, 108, 200.0, seed=int(rng.integers(1 << 20)), R=Rm, position=c))
    return cams


def eager(R, sc, cams):
    """Eager render; also returns the PBF pair count, which a plan's
    association capacity bounds."""
    rgb, depth, trans, frame = R.render(sc, cams, keep_frame=True)
    torch.cuda.synchronize()
    e = frame.stats()["n_candidates"]
    frame.release()
    return rgb, depth, trans, e


def test_plan_equals_eager_over_launches(R):
    scene = synth.scene_box(20000, seed=11, half=4.0)
    sc = R.scene_from_numpy(scene)
    rng = np.random.default_rng(0)
    shapes = small_cams(rng, [0, 2, 1])
    plan = R.Plan(sc, shapes, entry_capacity=2_000_000)
    for it in range(3):
        cams = small_cams(rng, [0, 2, 1])
        plan.launch(cams)
        E, cap, over = plan.entries()
        rgb, depth, trans, e = eager(R, sc, cams)
        assert not over and E == e and cap == 2_000_000
        assert torch.equal(plan.rgb, rgb) and torch.equal(plan.depth, depth) and torch.equal(plan.trans, trans), it
    # the camera model may change between launches, the grid size may not
    cams = small_cams(rng, [0, 2, 1])
    cams[0] = synth.camera_kb(80, 60, 190.0, seed=4, R=cams[0]["R"], position=-cams[0]["R"].T @ cams[0]["t"])
    plan.launch(cams)
    rgb, _, _, _ = eager(R, sc, cams)
    plan.entries()
    assert torch.equal(plan.rgb, rgb)
    with pytest.raises(_lib.GeerError):
        plan.launch(small_cams(rng, [1, 2, 1]))
    plan.destroy()


def test_plan_capacity_overflow_and_recovery(R):
    scene = synth.scene_box(20000, seed=12, half=4.0)
    sc = R.scene_from_numpy(scene)
    rng = np.random.default_rng(1)
    cams = small_cams(rng, [1, 1])
    rgb, depth, trans, e = eager(R, sc, cams)
    assert e > 100
    tight = R.Plan(sc, cams, entry_capacity=e - 1)
    tight.launch(cams)
    E, cap, over = tight.entries()
    assert over and E == e and cap == e - 1
    assert torch.all(tight.rgb == 0) and torch.all(tight.trans == 1) and torch.all(tight.depth == 0)
    # a batch that fits on the next launch renders correctly again
    other = small_cams(rng, [1, 1])
    rgb2, _, _, e2 = eager(R, sc, other)
    if e2 < e - 1:
        tight.launch(other)
        E2, _, over2 = tight.entries()
        assert not over2 and E2 == e2 and torch.equal(tight.rgb, rgb2)
    exact = R.Plan(sc, cams, entry_capacity=e)
    exact.launch(cams)
    assert not exact.entries()[2]
    assert torch.equal(exact.rgb, rgb) and torch.equal(exact.trans, trans)
    tight.destroy()
    exact.destroy()


def test_plan_workspace_and_invalid_arguments(R):
    scene = synth.scene_box(5000, seed=13, half=4.0)
    sc = R.scene_from_numpy(scene)
    cams = small_cams(np.random.default_rng(2), [0, 1])
    need = R.plan_workspace_bytes(sc, cams, 100_000)
    assert need > 5000 * 2 * 64
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    with pytest.raises(_lib.GeerError):
        R.Plan(sc, cams, 100_000, workspace=ws[off: off + need - 256])
    p = R.Plan(sc, cams, 100_000, workspace=ws[off: off + need])
    assert p.device_bytes() == 0
    p.launch(cams)
    rgb, _, _, _ = eager(R, sc, cams)
    p.entries()
    assert torch.equal(p.rgb, rgb)
    p.destroy()
    with pytest.raises(_lib.GeerError):
        R.Plan(sc, cams, 0)
    empty = R.scene_from_numpy(scene.subset(np.arange(0)))
    with pytest.raises(_lib.GeerError):
        R.Plan(empty, cams, 1000)


def served_vs_alone(R, sc, done):
    for r in done:
        rgb, depth, trans, _ = eager(R, sc, [r.cam])
        assert torch.equal(r.rgb, rgb) and torch.equal(r.depth, depth) and torch.equal(r.trans, trans), r.rid


def test_server_mix_equals_alone(R):
    from paper_2505_24053_amd import serve

    scene = synth.scene_box(30000, seed=14, half=4.0)
    sc = R.scene_from_numpy(scene)
    rng = np.random.default_rng(3)
    kinds = rng.integers(0, 3, 30)
    cams = small_cams(rng, kinds)
    shapes = {(c["width"], c["height"]) for c in cams}
    srv = serve.Server(sc, shapes, entries_per_tile=2000, slots=2, slot_views=2, max_views=3)
    assert srv.prepare(shapes) > 3
    reqs = [serve.Request(i, c) for i, c in enumerate(cams)]
    # a burst then a trickle: the burst forms multi-view batches, the rest
    # arrive while earlier batches are on the GPU
    arrivals = np.concatenate([np.zeros(12), 1e-3 * np.arange(1, 19)])
    done = srv.run(reqs, arrivals)
    assert sorted(r.rid for r in done) == list(range(30))
    assert srv.stats["views"] == 30 and srv.stats["batches"] < 30, srv.stats
    assert srv.stats["overlapped"] > 0, srv.stats
    assert srv.stats["overflows"] == 0
    served_vs_alone(R, sc, done)
    # one served request of each kind against the FP64 oracle on sampled rays
    for k in range(3):
        r = next(r for r in done if int(kinds[r.rid]) == k)
        w, h = r.shape
        pix = np.random.default_rng(k).choice(w * h, 256, replace=False)
        got = dict(rgb=r.rgb.view(3, -1).T.double().cpu().numpy(), depth=r.depth.double().cpu().numpy(),
                   trans=r.trans.double().cpu().numpy())
        compare_render(got, oracle.render(scene, r.cam, pix=pix), pix=pix)
    print("server stats", srv.stats, "overlap %.2f" % srv.device_overlap(), serve.latency_summary(done))
    srv.close()


def test_server_overflow_falls_back_to_eager(R):
    from paper_2505_24053_amd import serve

    scene = synth.scene_box(30000, seed=15, half=4.0)
    sc = R.scene_from_numpy(scene)
    rng = np.random.default_rng(4)
    cams = small_cams(rng, [0, 1, 2, 1, 0, 2])
    srv = serve.Server(sc, {(c["width"], c["height"]) for c in cams}, entries_per_tile=0.01, slots=2, max_views=2)
    done = srv.run([serve.Request(i, c) for i, c in enumerate(cams)])
    assert srv.stats["overflows"] > 0 and all(r.retried for r in done)
    served_vs_alone(R, sc, done)
    srv.close()


def test_server_full_size_requests(R):
    """1M Gaussians SH3 resident; one request of each serving class."""
    from paper_2505_24053_amd import serve

    scene = synth.scene_box(1_000_000, seed=0)
    sc = R.scene_from_numpy(scene)
    cams = synth.workload_serving_requests(3, seed=5)
    alone = [eager(R, sc, [c]) for c in cams]
    per_tile = max(a[3] / serve.tiles_of((c["width"], c["height"])) for a, c in zip(alone, cams))
    srv = serve.Server(sc, {(c["width"], c["height"]) for c in cams}, entries_per_tile=1.25 * per_tile, slots=2,
                       slot_views=2, max_views=2)
    done = srv.run([serve.Request(i, c) for i, c in enumerate(cams)])
    assert srv.stats["overflows"] == 0, srv.stats
    for r in done:
        rgb, depth, trans, _ = alone[r.rid]
        assert torch.equal(r.rgb, rgb) and torch.equal(r.depth, depth) and torch.equal(r.trans, trans), r.rid
    for r in done:
        w, h = r.shape
        pix = np.random.default_rng(r.rid).choice(w * h, 96, replace=False)
        got = dict(rgb=r.rgb.view(3, -1).T.double().cpu().numpy(), depth=r.depth.double().cpu().numpy(),
                   trans=r.trans.double().cpu().numpy())
        compare_render(got, oracle.render(scene, r.cam, pix=pix), pix=pix)
    print("full-size serving: entries per tile %.0f" % per_tile, srv.stats, serve.latency_summary(done))
    srv.close()


def test_server_saturated_full_size_three_slots(R):
    """Saturated serving at the full size: 1M Gaussians, three slots, every
    request queued at once, so the radix passes of different slots' plans run
    on the device together.  No batch may report a stalled sort, and every
    served result equals the same camera rendered alone."""
    from paper_2505_24053_amd import serve

    scene = synth.scene_box(1_000_000, seed=0)
    sc = R.scene_from_numpy(scene)
    cams = synth.workload_serving_requests(48, seed=9)
    alone = {}
    per_tile = 0.0
    for i, c in enumerate(cams[:6]):
        alone[i] = eager(R, sc, [c])
        per_tile = max(per_tile, alone[i][3] / serve.tiles_of((c["width"], c["height"])))
    srv = serve.Server(sc, {(c["width"], c["height"]) for c in cams}, entries_per_tile=2.0 * per_tile, slots=3,
                       slot_views=2, max_views=4)
    srv.prepare({(c["width"], c["height"]) for c in cams})
    done = srv.run([serve.Request(i, c) for i, c in enumerate(cams)])
    assert len(done) == len(cams)
    # (a batch over its capacity is re-rendered eagerly and still compared)
    assert srv.stats["stalls"] == 0, srv.stats
    assert srv.stats["overlapped"] > 0, srv.stats
    for r in done:
        if r.rid in alone:
            rgb, depth, trans, _ = alone[r.rid]
            assert torch.equal(r.rgb, rgb) and torch.equal(r.depth, depth) and torch.equal(r.trans, trans), r.rid
    print("saturated full-size serving", srv.stats, "overlap %.2f" % srv.device_overlap())
    srv.close()
