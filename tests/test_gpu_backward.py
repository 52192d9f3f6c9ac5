"""GPU parity of the hand-written adjoint (gs3_render_backward, through the
C-ABI) against FP64 autograd of the oracle.

For a seeded upstream gradient dF = dL/dfinal, L = sum(dF * final), every
gradient tensor of the GPU (raw scene parameters and both MLPs' weights)
is compared with torch float64 autograd of ``oracle.render`` at the same
inputs. Tolerance: |g_gpu - g_ref| <= 1e-4 * max(1, max |g_ref|) per tensor,
i.e. 1e-4 max abs at unit gradient scale, over every pixel and Gaussian:
the oracle's threshold decisions that float32 rounding may take either way
follow the GPU forward's (tests/parity_resolve.py), so its autograd is the
gradient of the function the GPU evaluated."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle.gs3_oracle import AMB_BUDGET
from paper_2410_11419_amd import synth
from parity_resolve import describe, resolve

pytestmark = pytest.mark.gpu

TOL = 1e-4

# oracle parameter layout (Gaussian first) -> library layout (Gaussian last)
_TO_LIB = {
    "mean": lambda x: x.T, "log_scale": lambda x: x.T, "rot": lambda x: x.T,
    "opacity_logit": lambda x: x, "shade_rot": lambda x: x.T, "albedo": lambda x: x.T,
    "lobe_axis": lambda x: x.permute(1, 2, 0), "lobe_log_sharp": lambda x: x.T,
    "lobe_amp": lambda x: x.permute(1, 2, 0), "feat": lambda x: x.T,
}


@pytest.fixture(scope="module")
def gs3():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2410_11419_amd import gs3 as g
    assert g.device_ok(), "libgs3 needs a gfx950 device"
    return g


def _oracle_grads(sc, cam, light, consts, use_mlps, dF, out_gpu):
    """FP64 autograd of L = sum(dF * final) through the oracle render whose
    float32-ambiguous threshold decisions follow the GPU forward's
    (tests/parity_resolve.py): the gradient of the very function the GPU
    evaluated, over every pixel and every Gaussian. Returns the gradients,
    the resolution counts and the forward outputs."""
    p = O.scene_tensors(sc, requires_grad=True)
    phi = psi = None
    if use_mlps:
        phi = [(torch.tensor(w, dtype=torch.float64, requires_grad=True),
                torch.tensor(b, dtype=torch.float64, requires_grad=True)) for w, b in sc.phi.layers]
        psi = [(torch.tensor(w, dtype=torch.float64, requires_grad=True),
                torch.tensor(b, dtype=torch.float64, requires_grad=True)) for w, b in sc.psi.layers]
    npx = cam.width * cam.height
    px = {k: out_gpu[k].cpu().numpy().reshape(-1, npx).squeeze(0) if out_gpu[k].dim() == 2 else
          out_gpu[k].cpu().numpy().reshape(3, npx) for k in ("final", "S", "Sh", "R", "T_final")}
    ref, info = resolve(sc, cam, light, consts, phi, psi, out_gpu["T"].cpu().numpy()[:sc.n], px, params=p)
    loss = (ref["final"] * torch.as_tensor(dF.reshape(3, -1), dtype=torch.float64)).sum()
    loss.backward()
    # a parameter the loss does not depend on (feat without MLPs) has no grad
    grads = {nm: _TO_LIB[nm](p[nm].grad if p[nm].grad is not None else torch.zeros_like(p[nm])).numpy()
             for nm in _TO_LIB}
    if use_mlps:
        for tag, m in (("phi", phi), ("psi", psi)):
            for i, (w, b) in enumerate(m):
                grads[f"{tag}_w{i}"] = w.grad.numpy()
                grads[f"{tag}_b{i}"] = b.grad.numpy()
    return grads, info, ref


def _gpu_grads(g, sc, cam, light, consts, use_mlps, dF):
    ds = g.DeviceScene.from_host(sc)
    rnd = g.Renderer(ds, consts, use_mlps=use_mlps)
    out = rnd.render(cam, light)
    out = {k: v.clone() for k, v in out.items()}
    dev = torch.as_tensor(dF, dtype=torch.float32).cuda().contiguous()
    gr = rnd.backward(cam, light, dev)
    torch.cuda.synchronize()
    res = {nm: v.cpu().numpy() for nm, v in gr.t.items()}
    if use_mlps:
        for tag, m in (("phi", gr.phi), ("psi", gr.psi)):
            for i, (w, b) in enumerate(m):
                res[f"{tag}_w{i}"] = w.cpu().numpy()
                res[f"{tag}_b{i}"] = b.cpu().numpy()
    return res, out


def _compare_grads(g, sc, cam, light, consts_o, consts_g, use_mlps, tag, seed=0):
    rng = np.random.default_rng(seed)
    dF = (rng.standard_normal((3, cam.height, cam.width)) / math.sqrt(cam.height * cam.width)).astype(np.float32)
    got, out = _gpu_grads(g, sc, cam, light, consts_g, use_mlps, dF)
    ref, info, fwd = _oracle_grads(sc, cam, light, consts_o, use_mlps, dF, out)
    # the outputs the oracle's error bound alone would have flagged
    amb_g = fwd["amb_T"].numpy() > AMB_BUDGET
    n_amb_px = int((fwd["amb_px"].detach().numpy() > AMB_BUDGET).sum())
    worst, worst_flagged = {}, {}
    for nm, r in ref.items():
        a = got[nm]
        assert a.shape == r.shape, (nm, a.shape, r.shape)
        scale = max(1.0, float(np.abs(r).max()) if r.size else 1.0)
        err = float(np.abs(a - r).max()) if r.size else 0.0
        worst[nm] = (err / scale, scale)
        if nm in _TO_LIB and amb_g.any():
            sel = (slice(None),) * (a.ndim - 1) + (amb_g,)
            worst_flagged[nm] = float(np.abs(a[sel] - r[sel]).max()) / scale
    print(f"[{tag}] gradient error / scale: " +
          ", ".join(f"{k} {e:.1e}/{s:.1e}" for k, (e, s) in worst.items()) +
          f"; {describe(info)}; bound-flagged Gaussians {int(amb_g.sum())}/{sc.n} (max error / scale "
          f"{max(worst_flagged.values(), default=0.0):.1e}), bound-flagged pixels {n_amb_px}")
    assert not info["unresolved_T"].any() and not info["unresolved_px"].any()
    for nm, (e, s) in worst.items():
        assert e <= TOL, (nm, e, s)
    # the gradients are not trivially zero
    assert np.abs(ref["mean"]).max() > 0 and np.abs(got["opacity_logit"]).max() > 0


def test_backward_gradcheck_scene(gs3):
    sc, cam, light = synth.scene_gradcheck(seed=0)
    _compare_grads(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "gradcheck")


def test_backward_smooth_mode(gs3):
    sc, cam, light = synth.scene_gradcheck(seed=1, n=160)
    kg = gs3.make_consts(dilation=0.0, cutoff=math.inf, alpha_min=0.0, alpha_max=1.0, t_min=0.0,
                         shadow_bias=0.0)
    _compare_grads(gs3, sc, cam, light, O.SMOOTH, kg, True, "smooth")


def test_backward_small_scene_no_mlps(gs3):
    sc, cam, light = synth.scene_small(seed=2)
    sub = synth.subset(sc, np.arange(2048))
    _compare_grads(gs3, sub, cam, light, O.Consts(), gs3.default_consts(), False, "small")


def test_backward_ragged_multibatch(gs3):
    # lists longer than one staged batch, ragged image edges, both MLPs
    sc = synth.make_scene(6000, 8, seed=7, means="shell", mlps=True, log_scale_mu=(-3.4,) * 3)
    rng = np.random.default_rng(3)
    cam = synth.make_view(rng.standard_normal(3), 4.0, 120, 88, 40.0)
    light = synth.make_view(rng.standard_normal(3), 4.0, 136, 136, 40.0)
    _compare_grads(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "ragged")


def test_backward_fluffy(gs3):
    # the dense scene's distributions (70 % low-opacity needles in the cube,
    # 30 % shell) at a size the oracle's autograd finishes: long lists, rays
    # that stay lit through many splats, light splat at 60 deg
    sc = synth.make_scene(8000, 8, seed=13, means="shell", mlps=True, fluffy_fraction=0.7)
    rng = np.random.default_rng(13)
    cam = synth.make_view(rng.standard_normal(3), 4.0, 96, 72, 40.0)
    light = synth.make_view(rng.standard_normal(3), 4.0, 128, 128, 60.0)
    _compare_grads(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "fluffy")


def test_backward_banded_needles(gs3):
    # the denominator adjoint's banded path: needles spanning 16+ light
    # tiles with a bounding box several times their ellipse
    from test_gpu_parity import banded_count
    sc, cam, light = synth.scene_needles(seed=1)
    nb = banded_count(sc, light)
    print(f"[needles] {nb} banded splats in the light view")
    assert nb >= 10
    _compare_grads(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "needles")


def test_backward_accumulates(gs3):
    # two backward calls into one gradient buffer add up
    sc, cam, light = synth.scene_gradcheck(seed=5, n=128)
    ds = gs3.DeviceScene.from_host(sc)
    rnd = gs3.Renderer(ds)
    rnd.render(cam, light)
    dF = torch.randn(3, cam.height, cam.width, generator=torch.Generator().manual_seed(0)).cuda()
    g1 = rnd.backward(cam, light, dF)
    once = {k: v.clone() for k, v in g1.t.items()}
    rnd.backward(cam, light, dF, g1)
    for k, v in g1.t.items():
        assert torch.allclose(v, 2 * once[k], rtol=1e-5, atol=1e-7), k


def test_autograd_function(gs3):
    # RelitRender behind torch.autograd: leaf-tensor .grad equals the direct call
    sc, cam, light = synth.scene_gradcheck(seed=6, n=96)
    ds = gs3.DeviceScene.from_host(sc)
    for t in gs3.scene_parameters(ds):
        t.requires_grad_(True)
    rnd = gs3.Renderer(ds)
    final = gs3.relit_render(rnd, cam, light)
    target = torch.zeros_like(final)
    loss = (final - target).abs().sum()
    loss.backward()
    dF = torch.sign(final.detach() - target)
    rnd2 = gs3.Renderer(ds)
    rnd2.render(cam, light)
    direct = rnd2.backward(cam, light, dF)
    for k, v in direct.t.items():
        assert torch.allclose(ds.t[k].grad, v, rtol=1e-5, atol=1e-6), k
    assert torch.allclose(ds.phi[0][0].grad, direct.phi[0][0], rtol=1e-5, atol=1e-6)
