"""GPU parity of the paper's own appearance model and MLP form (shared
anisotropic basis angular Gaussians, Sec. 4.1; Phi {32}^3 and Psi {128}^3
with positional encoding, latent and leaky ReLU, Sec. 4.2-4.3) against the
FP64 oracle, through the C-ABI.

- full renders (small cube scene with a point light, the same moved far
  from the origin, a ragged shell scene with a directional light): shadow
  values, per-Gaussian c, T', r and every pixel of every image within 1e-4,
  flagged threshold decisions resolved as in the other parity tests;
- per-Gaussian c, T', r of all 300,000 Gaussians of the full-size basis
  scene (camera 800^2, light 1024^2), with the GPU's T as Phi's input;
- the MLPs over hidden activations rescaled by 1e-3 and 1e3 (a
  function-preserving rescaling of the layers) and over tiny inputs;
- every gradient of the adjoint (scene parameters, shared basis, latent,
  both MLPs) against FP64 autograd of the oracle, point and directional
  light, within 1e-4 of each tensor's scale.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2410_11419_amd import synth
from parity_resolve import describe, resolve
from test_gpu_parity import _compare_render

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def gs3():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2410_11419_amd import gs3 as g
    assert g.device_ok(), "libgs3 needs a gfx950 device"
    return g


def test_basis_render_parity_small(gs3):
    sc, cam, light = synth.scene_basis_small()
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "basis_small")


def test_basis_render_parity_directional_ragged(gs3):
    sc = synth.make_basis_scene(9000, 3, means="shell", mlps=True, log_scale_mu=(-3.6,) * 3)
    rng = np.random.default_rng(4)
    cam = synth.make_view(rng.standard_normal(3), 4.0, 200, 152, 40.0)     # ragged tiles
    light = synth.make_directional(rng.standard_normal(3), 176, 176, 2.4)
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "basis_directional")


def test_basis_render_translated_scene(gs3):
    # the scene, camera and light moved far from the origin: the encoding of
    # mu then spans tens of turns per band (2^(j-1) mu), which the kernels
    # reduce to [-1/2, 1/2] turns before the hardware sine and cosine
    sc, cam, light = synth.scene_basis_small(seed=6, n=3000)
    off = np.array([24.5, -17.25, 11.0])
    sc.mean = (sc.mean + off[:, None]).astype(np.float32)
    cam = synth.View(eye=cam.eye + off, target=cam.target + off, width=cam.width, height=cam.height, fov=cam.fov)
    light = synth.View(eye=light.eye + off, target=light.target + off, width=light.width, height=light.height,
                       fov=light.fov)
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "basis_translated")


def test_basis_render_without_mlps(gs3):
    sc, cam, light = synth.scene_basis_small(seed=2, n=3000, mlps=False)
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), False, "basis_no_mlps")


@pytest.mark.parametrize("scale", [1e-3, 1e3])
def test_basis_mlp_activation_scale(gs3, scale):
    # leaky ReLU is positively homogeneous: scaling the first layer and the
    # hidden biases by s and the output layer by 1/s keeps the function while
    # the hidden activations become s times their size
    sc = synth.make_basis_scene(4096, 8, means="shell", mlps=True, log_scale_mu=(-3.6,) * 3)
    for mlp in (sc.phi, sc.psi):
        L = mlp.layers
        L[0] = ((L[0][0] * scale).astype(np.float32), (L[0][1] * scale).astype(np.float32))
        L[1] = (L[1][0], (L[1][1] * scale).astype(np.float32))
        L[2] = (L[2][0], (L[2][1] * scale).astype(np.float32))
        L[3] = ((L[3][0] / scale).astype(np.float32), L[3][1])
    rng = np.random.default_rng(2)
    cam = synth.make_view(rng.standard_normal(3), 4.0, 128, 128, 40.0)
    light = synth.make_view(rng.standard_normal(3), 4.0, 128, 128, 60.0)
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, f"basis_scale_{scale:g}")


def test_basis_full_size_per_gaussian(gs3):
    """c, T' and r of every Gaussian of the 300K basis scene (800^2 camera,
    1024^2 light): the oracle's shading and MLPs given the GPU's T."""
    sc, cam, light = synth.scene_basis_full()
    ds = gs3.DeviceScene.from_host(sc)
    rnd = gs3.Renderer(ds)
    out = rnd.render(cam, light)
    torch.cuda.synchronize()
    T_g = out["T"].cpu().numpy()[:sc.n].astype(np.float64)
    col = out["colour"].cpu().numpy()[:, :sc.n]
    print(f"[basis_full] T range {T_g.min():.3f}..{T_g.max():.3f}")
    p = O.scene_tensors(sc)
    with torch.no_grad():
        sh = O.shade_basis(p, light.eye, cam.eye)
        Tt = torch.as_tensor(T_g)
        xphi, xpsi = O.basis_mlp_inputs(p, Tt, sh["wi"], sh["wo"])
        tp = O.mlp_forward(sc.phi.layers, xphi, O.LEAKY_SLOPE)[:, 0].numpy()
        r = O.mlp_forward(sc.psi.layers, xpsi, O.LEAKY_SLOPE).numpy()
    c = sh["c"].numpy()
    err_c = np.abs(col[0:3] - c.T).max()
    err_tp = np.abs(col[3] - tp).max()
    err_r = np.abs(col[4:7] - r.T).max()
    print(f"[basis_full] 300000 Gaussians: c max|err| {err_c:.2e} (|c| <= {np.abs(c).max():.1f}), "
          f"T' {err_tp:.2e}, r {err_r:.2e}")
    assert err_c <= TOL and err_tp <= TOL and err_r <= TOL
    assert np.isfinite(out["final"].cpu().numpy()).all()


# ---------------------------------------------------------------- adjoint

_TO_LIB = {
    "mean": lambda x: x.T, "log_scale": lambda x: x.T, "rot": lambda x: x.T,
    "opacity_logit": lambda x: x, "shade_rot": lambda x: x.T, "albedo": lambda x: x.T,
    "spec_albedo": lambda x: x.T, "basis_weight": lambda x: x.T, "latent": lambda x: x.T,
    "basis_rot": lambda x: x, "basis_log_sigma": lambda x: x,
}


def _compare_basis_grads(g, sc, cam, light, use_mlps, tag, seed=0):
    consts_o, consts_g = O.Consts(), g.default_consts()
    rng = np.random.default_rng(seed)
    dF = (rng.standard_normal((3, cam.height, cam.width)) / math.sqrt(cam.height * cam.width)).astype(np.float32)
    ds = g.DeviceScene.from_host(sc)
    rnd = g.Renderer(ds, consts_g, use_mlps=use_mlps)
    out = {k: v.clone() for k, v in rnd.render(cam, light).items()}
    gr = rnd.backward(cam, light, torch.as_tensor(dF).cuda().contiguous())
    torch.cuda.synchronize()
    got = {nm: v.cpu().numpy() for nm, v in gr.t.items()}
    if use_mlps:
        for t, m in (("phi", gr.phi), ("psi", gr.psi)):
            for i, (w, b) in enumerate(m):
                got[f"{t}_w{i}"], got[f"{t}_b{i}"] = w.cpu().numpy(), b.cpu().numpy()
    # oracle autograd with the GPU's flagged decisions
    p = O.scene_tensors(sc, requires_grad=True)
    phi = psi = None
    if use_mlps:
        phi = [(torch.tensor(w, dtype=torch.float64, requires_grad=True),
                torch.tensor(b, dtype=torch.float64, requires_grad=True)) for w, b in sc.phi.layers]
        psi = [(torch.tensor(w, dtype=torch.float64, requires_grad=True),
                torch.tensor(b, dtype=torch.float64, requires_grad=True)) for w, b in sc.psi.layers]
    npx = cam.width * cam.height
    px = {k: out[k].cpu().numpy().reshape(-1, npx).squeeze(0) if out[k].dim() == 2 else
          out[k].cpu().numpy().reshape(3, npx) for k in ("final", "S", "Sh", "R", "T_final")}
    ref_out, info = resolve(sc, cam, light, consts_o, phi, psi, out["T"].cpu().numpy()[:sc.n], px, params=p)
    (ref_out["final"] * torch.as_tensor(dF.reshape(3, -1), dtype=torch.float64)).sum().backward()
    ref = {nm: f(p[nm].grad).numpy() for nm, f in _TO_LIB.items()}
    if use_mlps:
        for t, m in (("phi", phi), ("psi", psi)):
            for i, (w, b) in enumerate(m):
                ref[f"{t}_w{i}"], ref[f"{t}_b{i}"] = w.grad.numpy(), b.grad.numpy()
    worst = {}
    for nm, r in ref.items():
        a = got[nm]
        assert a.shape == r.shape, (nm, a.shape, r.shape)
        scale = max(1.0, float(np.abs(r).max()))
        worst[nm] = (float(np.abs(a - r).max()) / scale, scale)
    print(f"[{tag}] gradient error / scale: " + ", ".join(f"{k} {e:.1e}/{s:.1e}" for k, (e, s) in worst.items()) +
          f"; {describe(info)}")
    assert not info["unresolved_T"].any() and not info["unresolved_px"].any()
    for nm, (e, s) in worst.items():
        assert e <= TOL, (nm, e, s)
    assert np.abs(ref["basis_rot"]).max() > 0 and np.abs(got["latent"]).max() > 0


def test_basis_backward_gradcheck_scene(gs3):
    sc, cam, light = synth.scene_basis_gradcheck(seed=3)
    _compare_basis_grads(gs3, sc, cam, light, True, "basis_bwd")


def test_basis_backward_directional_light(gs3):
    sc, cam, light = synth.scene_basis_gradcheck(seed=5, n=300)
    light = synth.make_directional(light.eye, 40, 40, 2.6)
    _compare_basis_grads(gs3, sc, cam, light, True, "basis_bwd_dir", seed=1)


def test_basis_backward_ragged_many_gaussians(gs3):
    # several workgroups of every adjoint kernel, a ragged Gaussian count and
    # a ragged camera
    sc = synth.make_basis_scene(2999, 11, means="cube", mlps=True, log_scale_mu=(-2.6,) * 3,
                                log_scale_sd=(0.3,) * 3, k=5)
    rng = np.random.default_rng(8)
    cam = synth.make_view(rng.standard_normal(3), 4.0, 72, 56, 40.0)
    light = synth.make_view(rng.standard_normal(3), 4.0, 64, 64, 60.0)
    _compare_basis_grads(gs3, sc, cam, light, True, "basis_bwd_ragged", seed=2)
