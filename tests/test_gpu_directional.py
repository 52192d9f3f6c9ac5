"""GPU parity of directional and environment lighting (Sec. 4.5).

A directional light's shadow splat uses an orthographic light view; its
shading takes the light direction for every Gaussian. Forward outputs and
the hand-written adjoint are compared with the oracle exactly as for point
lights (float32-ambiguous decisions resolved to the GPU's outcome,
tests/parity_resolve.py; 1e-4 max abs). The environment render is the
weighted sum of the directional renders: the GPU's Renderer.render_env is
checked against the oracle's sum of resolved renders and against the sum of
the GPU's own single-light frames."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2410_11419_amd import synth
from test_gpu_backward import _compare_grads
from test_gpu_parity import TOL, _compare_render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs3():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2410_11419_amd import gs3 as g
    assert g.device_ok(), "libgs3 needs a gfx950 device"
    return g


def _dir(seed):
    return np.random.default_rng(seed).standard_normal(3)


def test_render_parity_directional_small(gs3):
    sc, cam, _ = synth.scene_small(seed=4)
    light = synth.make_directional(_dir(31), 160, 160, 3.6)
    print(f"light direction {light.eye / 4.0}")
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), False, "directional")


def test_render_parity_directional_mlps_ragged(gs3):
    # MLPs on, ragged camera and light images, a light that also reaches the
    # Gaussians the camera sees from behind
    sc = synth.make_scene(12000, 8, seed=15, means="shell", mlps=True, log_scale_mu=(-3.6,) * 3)
    rng = np.random.default_rng(5)
    cam = synth.make_view(rng.standard_normal(3), 4.0, 200, 152, 40.0)
    light = synth.make_directional(rng.standard_normal(3), 184, 136, 2.4)
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "directional_mlp")


def test_render_parity_directional_needles(gs3):
    # thin needles on the denominator's banded path under the orthographic
    # light view
    sc, cam, _ = synth.scene_needles(seed=2)
    light = synth.make_directional(_dir(33), 256, 256, 3.6)
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "directional_needles")


def test_backward_parity_directional(gs3):
    sc, cam, _ = synth.scene_gradcheck(seed=6)
    light = synth.make_directional(_dir(34), 40, 40, 3.6)
    _compare_grads(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "directional_bwd")


def test_backward_parity_directional_smooth(gs3):
    # every decision off: the adjoint of the orthographic projection itself
    sc, cam, _ = synth.scene_gradcheck(seed=7, n=160)
    light = synth.make_directional(_dir(35), 36, 36, 3.6)
    kg = gs3.make_consts(dilation=0.0, cutoff=float("inf"), alpha_min=0.0, alpha_max=1.0, t_min=0.0,
                         shadow_bias=0.0)
    _compare_grads(gs3, sc, cam, light, O.SMOOTH, kg, True, "directional_smooth")


def test_environment_render(gs3):
    """render_env of 6 sampled directional lights: within 1e-4 of the
    oracle's weighted sum of its resolved single-light renders, and within
    1e-6 of the weighted sum of the GPU's own single-light frames (the
    shadow numerator's float atomics may add in another order)."""
    sc, cam, _ = synth.scene_small(seed=5)
    lights, w = synth.environment_lights(6, seed=3, width=128, height=128, ortho_width=3.6)
    ds = gs3.DeviceScene.from_host(sc)
    rnd = gs3.Renderer(ds, use_mlps=False)
    env = rnd.render_env(cam, lights, w).cpu().numpy()
    own = np.zeros_like(env)
    ref = np.zeros((3, cam.height * cam.width))
    for i, (lv, wi) in enumerate(zip(lights, w)):
        out, r = _compare_render(gs3, sc, cam, lv, O.Consts(), gs3.default_consts(), False, f"env_light{i}",
                                 nonempty=False)
        own += np.float32(wi) * out["final"].cpu().numpy()
        ref += float(wi) * O.render_images(r, cam)["final"].reshape(3, -1)
    e_own = float(np.abs(env - own).max())
    e_ref = float(np.abs(env.reshape(3, -1) - ref).max())
    print(f"environment of {len(lights)} lights: |env - sum of GPU frames| {e_own:.2e}, "
          f"|env - oracle| {e_ref:.2e}, mean {env.mean():.3f}")
    assert e_own <= 1e-6
    assert e_ref <= TOL
    assert env.max() > 0.05


def test_environment_argument_checks(gs3):
    sc, cam, _ = synth.scene_small(seed=5)
    rnd = gs3.Renderer(gs3.DeviceScene.from_host(synth.subset(sc, np.arange(100))), use_mlps=False)
    lights, w = synth.environment_lights(2, seed=3, width=32, height=32, ortho_width=3.6)
    with pytest.raises(ValueError):
        rnd.render_env(cam, lights, w[:1])
    with pytest.raises(ValueError):
        rnd.render_env(cam, [], [])
    bad = synth.make_directional(_dir(1), 32, 32, 0.0)
    with pytest.raises(gs3.Gs3Error):
        rnd.render_env(cam, [bad], [1.0])


def test_environment_pipeline_equals_one_slot(gs3):
    """EnvPipeline with 4 lights in flight over 6 lights (slots of two and
    one light) equals render_env on one renderer within 1e-6 (only the
    order of the weighted additions differs), and gives the same bits on
    a second call."""
    sc, cam, _ = synth.scene_small(seed=6)
    lights, w = synth.environment_lights(6, seed=5, width=128, height=128, ortho_width=3.6)
    ds = gs3.DeviceScene.from_host(sc)
    one = gs3.Renderer(ds).render_env(cam, lights, w).clone()
    ep = gs3.EnvPipeline(ds, slots=4)
    a = ep.render(cam, lights, w).clone()
    b = ep.render(cam, lights, w, check=False).clone()
    torch.cuda.synchronize()
    err = float((a - one).abs().max())
    print(f"environment pipeline vs one slot: {err:.2e}")
    assert err <= 1e-6
    assert torch.equal(a, b)
