"""Pins of the oracle's shared-basis appearance model and MLP form.

The paper's own appearance (Sec. 4.1: a Lambertian plus a linear combination
of K basis angular Gaussians shared by all spatial Gaussians, anisotropic
Eq. 7) and its MLP form (Sec. 4.2 Eq. 8 and Sec. 4.3: positional encoding,
a 6-D latent, leaky ReLU, Phi {32}^3, Psi {128}^3) are checked here against
closed forms, invariants and library routines:

- the encoding against its values at exactly representable points;
- the basis shading against Eq. 7 written in spherical coordinates of the
  half vector in each basis frame (a different route from the oracle's
  projection onto the frame's x-y plane), with light and camera placed so
  that h' is known in closed form;
- invariance of the colour under a rotation of the world applied to the
  centre, the light, the camera and the shading frame together;
- the degenerate cases: zero weights (Lambertian only) and one isotropic
  basis (the per-Gaussian isotropic lobe of the configs' form);
- the MLPs against torch.nn with LeakyReLU;
- autograd of the whole render against float64 central differences.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import oracle as O
from paper_2410_11419_amd import synth

T = lambda a: torch.as_tensor(np.asarray(a, np.float64))  # noqa: E731


def test_positional_encoding_closed_form():
    x = T([[0.0, 0.25, 0.5]])
    pe = O.positional_encoding(x).numpy()[0]
    assert pe.shape == (27,)
    r2 = math.sqrt(0.5)
    expect = [0.0, 0.25, 0.5,
              0.0, r2, 1.0, 1.0, r2, 0.0,            # sin(pi x), cos(pi x)
              0.0, 1.0, 0.0, 1.0, 0.0, -1.0,         # sin(2 pi x), cos(2 pi x)
              0.0, 0.0, 0.0, 1.0, -1.0, 1.0,         # sin(4 pi x), cos(4 pi x)
              0.0, 0.0, 0.0, 1.0, 1.0, 1.0]          # sin(8 pi x), cos(8 pi x)
    np.testing.assert_allclose(pe, expect, atol=1e-14)
    # sin^2 + cos^2 = 1 in every band, for arbitrary inputs
    y = torch.randn(5, 3, dtype=torch.float64)
    p = O.positional_encoding(y)
    for k in range(O.PE_BANDS):
        s, c = p[:, 3 + 6 * k: 6 + 6 * k], p[:, 6 + 6 * k: 9 + 6 * k]
        np.testing.assert_allclose((s * s + c * c).numpy(), 1.0, rtol=1e-14)
        np.testing.assert_allclose(s.numpy(), np.sin(2 ** k * np.pi * y.numpy()), rtol=1e-13, atol=1e-15)


def _basis_scene(n, k, seed):
    sc = synth.make_basis_scene(n, seed, k=k, mlps=False)
    return sc


def _eq7_spherical(h_local, sx, sy, sz):
    """Eq. 7 with h' given in the basis frame by its polar angle theta (from
    z) and azimuth phi (from x toward y):
    G = exp(-theta^2 (cos^2 phi / sx^2 + sin^2 phi / sy^2) / (2 sz^2)) / sz."""
    a, b, c = h_local
    theta = math.acos(max(-1.0, min(1.0, c)))
    phi = math.atan2(b, a)
    e = theta ** 2 * (math.cos(phi) ** 2 / sx ** 2 + math.sin(phi) ** 2 / sy ** 2) / sz ** 2
    return math.exp(-0.5 * e) / sz


def test_basis_shading_eq4_to_7_closed_form():
    # light and camera at the same point: w_i = w_o, so h' = w_i' and the
    # colour is rho_d f_d(h'_z) + rho_s sum_j alpha_j G_j(R_j h')
    n, k = 40, 5
    sc = _basis_scene(n, k, 11)
    p = O.scene_tensors(sc)
    pos = np.array([0.7, -2.9, 2.2])
    out = O.shade_basis(p, pos, pos)
    mu = sc.mean.T.astype(np.float64)
    w = pos - mu
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    qs = sc.shade_rot.T.astype(np.float64)
    Rsh = Rotation.from_quat(np.concatenate([qs[:, 1:], qs[:, :1]], 1)).as_matrix()   # scipy: x, y, z, w
    qb = sc.basis.basis_rot.astype(np.float64)
    Rb = Rotation.from_quat(np.concatenate([qb[:, 1:], qb[:, :1]], 1)).as_matrix()
    sig = np.exp(sc.basis.basis_log_sigma.astype(np.float64))
    kd = 0.01 * (1 - math.exp(-1))
    for i in range(n):
        h = Rsh[i] @ w[i]
        cz = h[2]
        elu = cz if cz > 0 else 0.01 * (math.exp(cz) - 1)
        fd = (elu + kd) / ((1 + kd) * math.pi)
        fs = sum(float(sc.basis.weight[j, i]) * _eq7_spherical(Rb[j] @ h, *sig[j]) for j in range(k))
        ref = sc.albedo[:, i].astype(np.float64) * fd + sc.basis.spec_albedo[:, i].astype(np.float64) * fs
        np.testing.assert_allclose(out["c"][i].numpy(), ref, rtol=1e-10, atol=1e-14)


def test_basis_shading_rotation_invariance():
    # rotating the world (centres, light, camera) by M and every shading
    # frame by M^T (world -> shading becomes R_sh M^T) leaves every local
    # direction, hence the colour, unchanged
    sc = _basis_scene(30, 8, 12)
    p = O.scene_tensors(sc)
    light, eye = np.array([1.0, 3.0, -2.0]), np.array([-3.5, 0.4, 1.9])
    c0 = O.shade_basis(p, light, eye)["c"]
    M = Rotation.from_euler("zyx", [0.7, -0.4, 1.9])
    q = p["shade_rot"].numpy()
    rq = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1)) * M.inv()
    xyzw = rq.as_quat()
    p2 = dict(p)
    p2["shade_rot"] = T(np.concatenate([xyzw[:, 3:], xyzw[:, :3]], 1))
    p2["mean"] = T(M.apply(p["mean"].numpy()))
    c1 = O.shade_basis(p2, M.apply(light), M.apply(eye))["c"]
    np.testing.assert_allclose(c1.numpy(), c0.numpy(), rtol=1e-10, atol=1e-13)


def test_basis_shading_degenerate_cases():
    sc = _basis_scene(25, 3, 13)
    light, eye = np.array([2.0, -1.0, 3.0]), np.array([-1.0, 3.5, 0.5])
    # zero weights: the Lambertian term alone
    p = O.scene_tensors(sc)
    p["basis_weight"] = torch.zeros_like(p["basis_weight"])
    out = O.shade_basis(p, light, eye)
    wi = T(light) - p["mean"]
    wi = wi / torch.linalg.norm(wi, dim=1, keepdim=True)
    cos = (O.quat_to_rotmat(p["shade_rot"]) @ wi[..., None])[:, 2, 0]
    np.testing.assert_allclose(out["c"].numpy(), (p["albedo"] * O.diffuse(cos)[:, None]).numpy(), rtol=1e-13)
    # one basis with sigma_x = sigma_y = 1: the isotropic lobe lambda exp(-(lambda theta)^2 / 2)
    # with lambda = 1 / sigma_z, axis = the basis z, RGB amplitude alpha rho_s
    sc1 = _basis_scene(25, 1, 14)
    sc1.basis.basis_log_sigma[0, :2] = 0.0
    p = O.scene_tensors(sc1)
    out = O.shade_basis(p, light, eye)
    R = O.quat_to_rotmat(p["basis_rot"])[0]
    sz = math.exp(float(sc1.basis.basis_log_sigma[0, 2]))
    iso = dict(p)
    iso["lobe_axis"] = R[2].expand(25, 1, 3).clone()
    iso["lobe_log_sharp"] = torch.full((25, 1), -math.log(sz), dtype=torch.float64)
    iso["lobe_amp"] = (p["basis_weight"][:, :, None] * p["spec_albedo"][:, None, :])
    ref = O.shade(iso, light, eye)["c"]
    np.testing.assert_allclose(out["c"].numpy(), ref.numpy(), rtol=1e-10, atol=1e-14)


def test_basis_mlps_match_torch_nn():
    sc = synth.make_basis_scene(16, 4, k=2, mlps=True)
    assert sc.phi.n_in == 61 and sc.psi.n_in == 60
    assert [w.shape[0] for w, _ in sc.phi.layers] == [32, 32, 32, 1]
    assert [w.shape[0] for w, _ in sc.psi.layers] == [128, 128, 128, 3]
    for mlp in (sc.phi, sc.psi):
        x = torch.randn(64, mlp.n_in, dtype=torch.float64) * 2.0
        layers = []
        for i, (w, b) in enumerate(mlp.layers):
            lin = torch.nn.Linear(w.shape[1], w.shape[0]).double()
            with torch.no_grad():
                lin.weight.copy_(torch.as_tensor(w))
                lin.bias.copy_(torch.as_tensor(np.asarray(b, np.float64) + 0.05 * i))
            last = i + 1 == len(mlp.layers)
            layers += [lin, torch.nn.Sigmoid() if last else torch.nn.LeakyReLU(0.01)]
        ref = torch.nn.Sequential(*layers)(x)
        lay = [(w, np.asarray(b, np.float64) + 0.05 * i) for i, (w, b) in enumerate(mlp.layers)]
        np.testing.assert_allclose(O.mlp_forward(lay, x, O.LEAKY_SLOPE).detach().numpy(),
                                   ref.detach().numpy(), rtol=1e-13)


def test_basis_mlp_inputs_layout():
    # Phi gets [T, PE(w_i), PE(mu), l]; Psi gets [PE(w_o), PE(mu), l]
    sc = synth.make_basis_scene(7, 5, k=2, mlps=False)
    p = O.scene_tensors(sc)
    Tv = torch.rand(7, dtype=torch.float64)
    wi = torch.randn(7, 3, dtype=torch.float64)
    wo = torch.randn(7, 3, dtype=torch.float64)
    xphi, xpsi = O.basis_mlp_inputs(p, Tv, wi, wo)
    assert xphi.shape == (7, 61) and xpsi.shape == (7, 60)
    np.testing.assert_array_equal(xphi[:, 0].numpy(), Tv.numpy())
    np.testing.assert_array_equal(xphi[:, 1:4].numpy(), wi.numpy())
    np.testing.assert_array_equal(xphi[:, 28:31].numpy(), p["mean"].numpy())
    np.testing.assert_array_equal(xphi[:, 55:].numpy(), p["latent"].numpy())
    np.testing.assert_array_equal(xpsi[:, 0:3].numpy(), wo.numpy())
    np.testing.assert_array_equal(xpsi[:, 27:30].numpy(), p["mean"].numpy())
    np.testing.assert_array_equal(xpsi[:, 54:].numpy(), p["latent"].numpy())
    np.testing.assert_allclose(xpsi[:, 3:6].numpy(), np.sin(np.pi * wo.numpy()), rtol=1e-14)


BASIS_ENTRIES = [("mean", (3, 0)), ("log_scale", (4, 1)), ("opacity_logit", (2,)), ("shade_rot", (6, 2)),
                 ("albedo", (1, 1)), ("spec_albedo", (5, 2)), ("basis_weight", (8, 1)), ("latent", (9, 4)),
                 ("basis_rot", (1, 2)), ("basis_log_sigma", (0, 0)), ("basis_log_sigma", (1, 2)),
                 ("phi_w0", (7, 0)), ("phi_w0", (3, 40)), ("psi_w0", (5, 18)), ("psi_w2", (9, 100)),
                 ("phi_b3", (0,))]


@pytest.mark.parametrize("light_kind", ["point", "directional"])
def test_basis_autograd_matches_finite_differences(light_kind):
    sc, cam, light = synth.scene_basis_gradcheck(seed=31, n=20)
    sc.basis.basis_rot = sc.basis.basis_rot[:2].copy()
    sc.basis.basis_log_sigma = sc.basis.basis_log_sigma[:2].copy()
    sc.basis.weight = sc.basis.weight[:2].copy()
    cam = synth.View(cam.eye, cam.target, 14, 12, cam.fov)
    if light_kind == "point":
        light = synth.View(light.eye, light.target, 12, 12, light.fov)
    else:
        light = synth.make_directional(light.eye, 12, 12, 2.4)
    consts = O.SMOOTH
    rng = np.random.default_rng(32)
    wts = T(rng.standard_normal((3, 12 * 14)))
    phi0 = [(T(w), T(b)) for w, b in sc.phi.layers]
    psi0 = [(T(w), T(b)) for w, b in sc.psi.layers]

    def loss(p, phi, psi):
        return (O.render(sc, cam, light, consts, params=p, phi=phi, psi=psi)["final"] * wts).sum()

    p = O.scene_tensors(sc, requires_grad=True)
    phi = [(w.clone().requires_grad_(True), b.clone().requires_grad_(True)) for w, b in phi0]
    psi = [(w.clone().requires_grad_(True), b.clone().requires_grad_(True)) for w, b in psi0]
    L = loss(p, phi, psi)
    leaves = dict(p)
    leaves.update({"phi_w0": phi[0][0], "psi_w0": psi[0][0], "psi_w2": psi[2][0], "phi_b3": phi[3][1]})
    grads = dict(zip(leaves, torch.autograd.grad(L, list(leaves.values()), allow_unused=True)))
    for name, idx in BASIS_ENTRIES:
        base = leaves[name].detach().clone()

        def at(delta):
            q = {k: v.detach().clone() for k, v in p.items()}
            ph = [(w.detach().clone(), b.detach().clone()) for w, b in phi]
            ps = [(w.detach().clone(), b.detach().clone()) for w, b in psi]
            tgt = {"phi_w0": ph[0][0], "psi_w0": ps[0][0], "psi_w2": ps[2][0], "phi_b3": ph[3][1]}.get(name)
            tgt = q[name] if tgt is None else tgt
            tgt[idx] = base[idx] + delta
            with torch.no_grad():
                return loss(q, ph, ps).item()
        h = 1e-6
        fd = (at(h) - at(-h)) / (2 * h)
        an = grads[name][idx].item()
        assert an == pytest.approx(fd, rel=2e-4, abs=1e-6 * max(1.0, abs(L.item()))), (name, idx, an, fd)
