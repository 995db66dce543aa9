"""Host-side reporting of a stalled association sort.

Each radix pass waits on earlier blocks with a bounded spin; when it gives up
the forward's outputs are invalid.  Most of these tests set the flag word from
the host (geer_debug_mark_stalled) and check that every reporting path sees it
-- the next eager forward, geer_check, a frame's statistics, a plan's status --
and that the server re-renders such a batch.  One lowers the look-back limit
from the host (geer_debug_set_spin_limit) so that the passes give up for real,
with every kernel still ending, and checks that the damage is contained.
"""
import numpy as np
import pytest

from paper_2505_24053_amd import _lib, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_24053_amd import renderer

    return renderer


def mark_context(R):
    ctx = R.context(0)
    _lib.check(_lib.load().geer_debug_mark_stalled(ctx, None), ctx)


def test_eager_forward_reports_earlier_stall(R):
    scene, cams = synth.workload_small(seed=1)
    sc = R.scene_from_numpy(scene)
    ref, _, _, _ = R.render(sc, cams)
    torch.cuda.synchronize()
    mark_context(R)
    with pytest.raises(_lib.GeerError) as e:
        R.render(sc, cams)
    assert e.value.status == _lib.ERR_STALLED
    # reported once: the flag is cleared and rendering goes on
    again, _, _, _ = R.render(sc, cams)
    torch.cuda.synchronize()
    assert torch.equal(again, ref)
    R.check_errors()


def test_check_and_frame_stats_report_stall(R):
    scene, cams = synth.workload_small(seed=2)
    sc = R.scene_from_numpy(scene)
    mark_context(R)
    with pytest.raises(_lib.GeerError) as e:
        R.check_errors()
    assert e.value.status == _lib.ERR_STALLED
    R.check_errors()
    _, _, _, frame = R.render(sc, cams, keep_frame=True)
    frame.stats()
    mark_context(R)
    with pytest.raises(_lib.GeerError) as e:
        frame.stats()
    assert e.value.status == _lib.ERR_STALLED
    frame.stats()
    frame.release()


def test_plan_status_and_server_rerender(R):
    from paper_2505_24053_amd import serve

    scene = synth.scene_box(20_000, seed=3, half=4.0)
    sc = R.scene_from_numpy(scene)
    cams = synth.workload_serving_requests(3, seed=5)
    cams = [dict(c, width=c["width"] // 8, height=c["height"] // 8) for c in cams]
    plan = R.Plan(sc, [cams[0]], entry_capacity=2_000_000)
    plan.launch([cams[0]])
    assert not plan.status()["stalled"]
    plan.mark_stalled()
    st = plan.status()
    assert st["stalled"] and not st["overflow"]
    with pytest.raises(_lib.GeerError) as e:
        plan.entries()
    assert e.value.status == _lib.ERR_STALLED
    plan.launch([cams[0]])  # a new launch reads back fresh counters
    assert not plan.status()["stalled"]
    plan.destroy()

    srv = serve.Server(sc, {(c["width"], c["height"]) for c in cams}, entries_per_tile=400.0, slots=2, max_views=2)
    launch = srv.launch

    def launch_and_stall(slot, batch, now):
        launch(slot, batch, now)
        slot.plan.mark_stalled()

    srv.launch = launch_and_stall
    reqs = [serve.Request(i, c) for i, c in enumerate(cams)]
    done = srv.run(reqs)
    assert len(done) == 3 and all(r.retried for r in done)
    assert srv.stats["stalls"] == srv.stats["batches"] > 0
    for r in done:
        alone, d, t, _ = R.render(sc, [r.cam])
        torch.cuda.synchronize()
        assert torch.equal(r.rgb, alone) and torch.equal(r.depth, d) and torch.equal(r.trans, t)
    srv.close()


def test_forced_stall_is_contained(R):
    """A look-back limit of zero polls (set from the host) makes the radix
    passes of an eager forward give up for real, while every kernel still
    ends.  A pass that gives up leaves its output unordered: the frame must
    then come back as background (every tile range emptied) and the stall be
    reported; if no pass had to wait, the frame is the ordinary one.  The
    next forward at the default limit renders as before."""
    scene, cams = synth.workload_fisheye_forward(seed=4)
    sc = R.scene_from_numpy(scene)
    ref, ref_d, ref_t, _ = R.render(sc, cams)
    torch.cuda.synchronize()
    ctx = R.context(0)
    L = _lib.load()
    _lib.check(L.geer_debug_set_spin_limit(ctx, 0), ctx)
    try:
        rgb, depth, trans, _ = R.render(sc, cams)
        torch.cuda.synchronize()
    finally:
        _lib.check(L.geer_debug_set_spin_limit(ctx, -1), ctx)
    try:
        R.check_errors()
        stalled = False
    except _lib.GeerError as e:
        assert e.status == _lib.ERR_STALLED
        stalled = True
    if stalled:
        assert not bool(rgb.any()) and not bool(depth.any()) and bool((trans == 1.0).all())
    else:
        assert torch.equal(rgb, ref) and torch.equal(depth, ref_d) and torch.equal(trans, ref_t)
    print("forced stall:", stalled)
    again, d2, t2, _ = R.render(sc, cams)
    torch.cuda.synchronize()
    R.check_errors()
    assert torch.equal(again, ref) and torch.equal(d2, ref_d) and torch.equal(t2, ref_t)
