"""The training step on the GPU against the oracle: the fused Adam kernel
(activations, moments, bias correction, statistics) over several steps, the
refinement (decisions bit for bit, outputs to rounding), and a short
training run whose loss falls."""
import math

import numpy as np
import pytest

import oracle
from paper_2505_24053_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("mean", "scale", "quat", "opacity", "sh")


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_24053_amd import train

    return train


def state_np(n, deg, seed):
    rng = np.random.default_rng(seed)
    R = oracle.train_rows(deg)
    raw = rng.normal(0, 1, (R, n))
    raw[3:6] = rng.uniform(-4, -1, (3, n))
    raw[10] = rng.uniform(-6, 4, n)
    return raw.astype(np.float32)


def test_adam_matches_oracle(T):
    deg, n = 3, 5000
    raw0 = state_np(n, deg, 1)
    st = T.TrainState(torch.as_tensor(raw0, device="cuda"), deg)
    s_o, o_o = oracle.activate(raw0)
    np.testing.assert_allclose(st.scale.cpu().numpy(), s_o, rtol=2e-6)
    np.testing.assert_allclose(st.opacity.cpu().numpy(), o_o, rtol=2e-6, atol=1e-7)
    rng = np.random.default_rng(2)
    raw, m, v = raw0.astype(np.float64), np.zeros((raw0.shape[0], n)), np.zeros((raw0.shape[0], n))
    acc, cnt = np.zeros(n), np.zeros(n)
    lr = (1.6e-3, 5e-3, 1e-3, 5e-2, 2.5e-3)
    for t in range(1, 4):
        g = {k: a.astype(np.float32) for k, a in dict(
            mean=rng.normal(size=(3, n)), scale=rng.normal(size=(3, n)), quat=rng.normal(size=(4, n)),
            opacity=rng.normal(size=n), sh=rng.normal(size=(48, n))).items()}
        g["mean"][:, :100] = 0.0  # unseen Gaussians: no statistics
        st.adam_step({k: torch.as_tensor(a, device="cuda") for k, a in g.items()}, t, lr=lr, eps=1e-8)
        # the oracle starts each step from the GPU's FP32 state, so FP32
        # rounding does not compound
        ref = oracle.adam_step(raw, m, v, g, t, lr, eps=1e-8, accum=acc, count=cnt)
        got_raw = st.raw.double().cpu().numpy()
        scale = np.abs(ref["raw"] - raw).max()
        assert np.abs(got_raw - ref["raw"]).max() <= 1e-6 + 1e-5 * scale
        np.testing.assert_allclose(st.m.double().cpu().numpy(), ref["m"], rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(st.v.double().cpu().numpy(), ref["v"], rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(st.accum.double().cpu().numpy(), ref["accum"], rtol=1e-5)
        np.testing.assert_array_equal(st.count.cpu().numpy(), ref["count"])
        s_o, o_o = oracle.activate(got_raw)
        np.testing.assert_allclose(st.scale.double().cpu().numpy(), s_o, rtol=2e-6)
        np.testing.assert_allclose(st.opacity.double().cpu().numpy(), o_o, rtol=2e-6, atol=1e-7)
        raw, m, v = got_raw, st.m.double().cpu().numpy(), st.v.double().cpu().numpy()
        acc, cnt = st.accum.double().cpu().numpy(), st.count.double().cpu().numpy()


def test_densify_matches_oracle(T):
    deg, n = 1, 20000
    raw = state_np(n, deg, 3)
    rng = np.random.default_rng(4)
    st = T.TrainState(torch.as_tensor(raw, device="cuda"), deg)
    st.m.copy_(torch.as_tensor(rng.normal(size=raw.shape).astype(np.float32)))
    st.v.copy_(torch.as_tensor(rng.uniform(0, 1, raw.shape).astype(np.float32)))
    st.accum.copy_(torch.as_tensor(rng.uniform(0, 0.01, n).astype(np.float32)))
    st.count.copy_(torch.as_tensor(rng.integers(0, 20, n).astype(np.float32)))
    noise = rng.normal(size=(6, n)).astype(np.float32)
    opts = dict(grad_threshold=2e-3, split_scale=0.1, min_opacity=0.01)
    out = st.densify(torch.as_tensor(noise, device="cuda"), **opts)
    torch.cuda.synchronize()
    ref = oracle.densify(raw, st.m.cpu().numpy(), st.v.cpu().numpy(), st.accum.cpu().numpy(), st.count.cpu().numpy(),
                         noise, **opts)
    kinds = np.bincount(ref["kinds"], minlength=4)
    assert (kinds > 100).all(), kinds  # every decision occurs
    assert out.n == ref["raw"].shape[1]
    got = out.raw.double().cpu().numpy()
    np.testing.assert_allclose(got, ref["raw"], rtol=1e-6, atol=1e-6)
    np.testing.assert_array_equal(out.m.cpu().numpy(), ref["m"].astype(np.float32))
    np.testing.assert_array_equal(out.v.cpu().numpy(), ref["v"].astype(np.float32))
    assert (out.accum == 0).all() and (out.count == 0).all()
    np.testing.assert_allclose(out.scale.double().cpu().numpy(), ref["scale"], rtol=2e-6)


def test_training_reduces_the_loss(T):
    """Fit a perturbed copy of a scene to renders of the original through a
    pinhole and a fisheye view: forward, L1, backward and Adam on the GPU,
    with one refinement half-way; the loss falls by a clear margin."""
    from paper_2505_24053_amd import renderer

    truth = synth.scene_box(3000, seed=6, half=3.0, sh_degree=1)
    start = synth.perturb(truth, 7)
    start.mean += np.random.default_rng(8).normal(0, 0.05, start.mean.shape).astype(np.float32)
    rng = np.random.default_rng(9)
    cams = [synth.camera_pinhole(96, 72, 70.0, *synth.random_pose(rng, 1.0)),
            synth.camera_equidistant(96, 96, 180.0, *synth.random_pose(rng, 1.0))]
    tsc = renderer.scene_from_numpy(truth)
    targets = [renderer.render(tsc, [c])[0] for c in cams]
    masks = [torch.ones(c["width"] * c["height"], dtype=torch.uint8, device="cuda") for c in cams]
    st = T.TrainState.from_scene(start)
    losses = []
    for it in range(1, 61):
        total = 0.0
        grads = {k: torch.zeros_like(st.scene()[k]) for k in KEYS}
        for c, tgt, mk in zip(cams, targets, masks):
            rgb, _, _, frame = renderer.render(st.scene(), [c], keep_frame=True)
            loss, dl = renderer.l1_loss(rgb, tgt, mk)
            renderer.backward(frame, st.scene(), dl / len(cams), accumulate=True, grads=grads)
            frame.release()
            total += float(loss.item()) / len(cams)
        losses.append(total)
        st.adam_step(grads, it, lr=(1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3))
        if it == 30:
            noise = torch.randn(6, st.n, generator=torch.Generator(device="cuda").manual_seed(1), device="cuda")
            st = st.densify(noise, grad_threshold=1e-6, split_scale=0.2, min_opacity=0.005)
    print("loss %.5f -> %.5f, %d Gaussians" % (losses[0], losses[-1], st.n))
    assert losses[-1] < 0.6 * losses[0]
