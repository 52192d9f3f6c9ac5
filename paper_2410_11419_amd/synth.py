"""Seeded synthetic inputs for the triple-splatting path.

This module only draws random numbers and packs them into arrays. It holds
none of the method's arithmetic (no projection, shading, splatting or MLP
evaluation), so both the HIP path and the CPU oracle may take their inputs
from it.

The paper's own scenes (trained Gaussians for NeRF-synthetic, NRHints and
lightstage captures, Sec. 5) are not available; these seeded scenes stand in
for them with the Gaussian counts, scale, opacity and appearance-parameter
distributions of the workloads the path is benchmarked on.

Draw order (all in float64 from ``numpy.random.default_rng(seed)``, cast to
float32 at the end, so the float32 arrays are the canonical input):
means, log-scales, rotation quaternions, opacity logits, albedo, lobe axes,
lobe log-sharpness, lobe amplitudes, shading quaternions, features, then the
two MLPs (Xavier-uniform weights, zero biases, layer order). Views come from
a second generator (seed 1 by default): a direction N(0,1)^3, normalised and
scaled to the view radius.

Layout is structure-of-arrays with the Gaussian index last (``[C, N]``), the
layout the library consumes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Scene", "View", "Mlp", "make_scene", "make_view", "random_views",
    "scene_small", "scene_full", "scene_fluffy", "fluffy_pairs", "scene_gradcheck",
    "perturb_scene", "subset", "concat_scenes", "scene_needles", "make_directional", "environment_lights",
    "BasisAppearance", "make_basis_scene", "scene_basis_small", "scene_basis_full", "scene_basis_gradcheck",
]

FEAT_DIM = 16
HIDDEN = 64
# the paper's MLP form (Sec. 4.2 / 4.3): 6-D latent, 4-band positional
# encoding of 3-vectors (3 + 2 * 4 * 3 = 27 values), Phi {32}^3, Psi {128}^3
LATENT_DIM = 6
PE_DIM = 27
PHI_BASIS_IN = 1 + 2 * PE_DIM + LATENT_DIM     # [T, PE(w_i), PE(mu), l]
PSI_BASIS_IN = 2 * PE_DIM + LATENT_DIM         # [PE(w_o), PE(mu), l]
PHI_BASIS_HIDDEN = 32
PSI_BASIS_HIDDEN = 128


@dataclasses.dataclass
class Mlp:
    """Dense MLP weights: ``layers[i] = (W [out, in], b [out])``."""
    layers: List[Tuple[np.ndarray, np.ndarray]]

    @property
    def n_in(self) -> int:
        return self.layers[0][0].shape[1]

    @property
    def n_out(self) -> int:
        return self.layers[-1][0].shape[0]


@dataclasses.dataclass
class BasisAppearance:
    """The paper's appearance parameters (Sec. 4.1 shared basis; Sec. 4.2
    latent): per Gaussian rho_s, basis weights alpha_j and the 6-D latent;
    shared by all Gaussians, the K basis angular Gaussians' frames and
    log-sigmas."""
    spec_albedo: np.ndarray      # [3, N]  rho_s
    weight: np.ndarray           # [K, N]  alpha_j
    latent: np.ndarray           # [6, N]  l
    basis_rot: np.ndarray        # [K, 4]  quaternion (w, x, y, z): shading -> basis frame
    basis_log_sigma: np.ndarray  # [K, 3]  log sigma_x, sigma_y, sigma_z

    @property
    def k(self) -> int:
        return self.weight.shape[0]


@dataclasses.dataclass
class Scene:
    """Raw (pre-activation) per-Gaussian parameters, float32 SoA."""
    mean: np.ndarray            # [3, N]
    log_scale: np.ndarray       # [3, N]
    rot: np.ndarray             # [4, N]  quaternion (w, x, y, z), any norm
    opacity_logit: np.ndarray   # [N]
    shade_rot: np.ndarray       # [4, N]  world -> shading frame quaternion
    albedo: np.ndarray          # [3, N]
    lobe_axis: np.ndarray       # [K, 3, N] (shading frame, any norm)
    lobe_log_sharp: np.ndarray  # [K, N]
    lobe_amp: np.ndarray        # [K, 3, N]
    feat: np.ndarray            # [16, N]
    phi: Optional[Mlp] = None   # shadow refinement MLP, None = passthrough
    psi: Optional[Mlp] = None   # residual RGB MLP, None = zero residual
    # the paper's shared-basis appearance; None = per-Gaussian isotropic lobes
    basis: Optional[BasisAppearance] = None

    @property
    def n(self) -> int:
        return self.mean.shape[1]

    @property
    def k(self) -> int:
        """Lobes per Gaussian, or basis angular Gaussians of a basis scene."""
        return self.basis.k if self.basis is not None else self.lobe_axis.shape[0]


@dataclasses.dataclass
class View:
    """View looking at ``target``: a pinhole (``fov`` horizontal, radians)
    or, with projection "orthographic", a parallel projection whose image
    spans ``ortho_width`` world units across (a directional light)."""
    eye: np.ndarray      # [3] float64
    target: np.ndarray   # [3] float64
    width: int
    height: int
    fov: float
    projection: str = "perspective"
    ortho_width: float = 0.0


def _unit_rows(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _xavier(rng: np.random.Generator, fan_in: int, fan_out: int):
    a = math.sqrt(6.0 / (fan_in + fan_out))
    w = rng.uniform(-a, a, size=(fan_out, fan_in))
    b = np.zeros(fan_out)
    return w, b


def _make_mlp(rng, n_in: int, n_out: int, hidden: int = HIDDEN, depth: int = 3) -> Mlp:
    dims = [n_in] + [hidden] * depth + [n_out]
    layers = []
    for i in range(len(dims) - 1):
        w, b = _xavier(rng, dims[i], dims[i + 1])
        layers.append((w.astype(np.float32), b.astype(np.float32)))
    return Mlp(layers)


def make_scene(n: int, k: int, seed: int = 0, *, means: str = "cube",
               log_scale_mu=(-4.0, -4.0, -4.0), log_scale_sd=(0.5, 0.5, 0.5),
               opacity_mu: float = 0.0, opacity_sd: float = 1.0,
               mlps: bool = False, fluffy_fraction: float = 0.0) -> Scene:
    """Draw one scene.

    means: "cube" = U[-1,1]^3; "shell" = unit direction times U[0.8, 1].
    fluffy_fraction: leading fraction of Gaussians drawn as a low-opacity,
    needle-shaped volume in U[-1,1]^3 (opacity logit N(-2,1), log-scales
    N(-2,.5), N(-5,.5), N(-5,.5)); the rest follow the other arguments.
    """
    rng = np.random.default_rng(seed)
    nf = int(round(n * fluffy_fraction))
    ns = n - nf
    # means
    parts = []
    if nf:
        parts.append(rng.uniform(-1.0, 1.0, size=(nf, 3)))
    if means == "cube":
        parts.append(rng.uniform(-1.0, 1.0, size=(ns, 3)))
    elif means == "shell":
        d = _unit_rows(rng.standard_normal((ns, 3)))
        r = rng.uniform(0.8, 1.0, size=(ns, 1))
        parts.append(d * r)
    else:
        raise ValueError(means)
    mean = np.concatenate(parts, 0)
    # log-scales
    ls = []
    if nf:
        ls.append(rng.normal((-2.0, -5.0, -5.0), (0.5, 0.5, 0.5), size=(nf, 3)))
    ls.append(rng.normal(log_scale_mu, log_scale_sd, size=(ns, 3)))
    log_scale = np.concatenate(ls, 0)
    rot = _unit_rows(rng.standard_normal((n, 4)))
    ol = []
    if nf:
        ol.append(rng.normal(-2.0, 1.0, size=nf))
    ol.append(rng.normal(opacity_mu, opacity_sd, size=ns))
    opacity_logit = np.concatenate(ol, 0)
    albedo = rng.uniform(0.0, 1.0, size=(n, 3))
    lobe_axis = _unit_rows(rng.standard_normal((n, k, 3)))
    lobe_log_sharp = rng.normal(2.0, 0.5, size=(n, k))
    lobe_amp = rng.uniform(0.0, 0.5, size=(n, k, 3))
    shade_rot = _unit_rows(rng.standard_normal((n, 4)))
    feat = rng.normal(0.0, 0.1, size=(n, FEAT_DIM))
    phi = psi = None
    if mlps:
        phi = _make_mlp(rng, 1 + FEAT_DIM, 1)
        psi = _make_mlp(rng, FEAT_DIM + 6, 3)
    f = np.float32
    return Scene(
        mean=np.ascontiguousarray(mean.T, f),
        log_scale=np.ascontiguousarray(log_scale.T, f),
        rot=np.ascontiguousarray(rot.T, f),
        opacity_logit=np.ascontiguousarray(opacity_logit, f),
        shade_rot=np.ascontiguousarray(shade_rot.T, f),
        albedo=np.ascontiguousarray(albedo.T, f),
        lobe_axis=np.ascontiguousarray(lobe_axis.transpose(1, 2, 0), f),
        lobe_log_sharp=np.ascontiguousarray(lobe_log_sharp.T, f),
        lobe_amp=np.ascontiguousarray(lobe_amp.transpose(1, 2, 0), f),
        feat=np.ascontiguousarray(feat.T, f),
        phi=phi, psi=psi,
    )


def make_view(direction, radius: float, width: int, height: int, fov_deg: float,
              target=(0.0, 0.0, 0.0)) -> View:
    d = np.asarray(direction, np.float64)
    d = d / np.linalg.norm(d)
    return View(eye=d * radius, target=np.asarray(target, np.float64),
                width=int(width), height=int(height), fov=math.radians(fov_deg))


def make_directional(direction, width: int, height: int, ortho_width: float, radius: float = 4.0) -> View:
    """A directional light shining from `direction` toward the origin: an
    orthographic view whose eye sits at `radius` along the direction."""
    d = np.asarray(direction, np.float64)
    d = d / np.linalg.norm(d)
    return View(eye=d * radius, target=np.zeros(3), width=int(width), height=int(height), fov=0.0,
                projection="orthographic", ortho_width=float(ortho_width))


def environment_lights(count: int, seed: int, width: int, height: int, ortho_width: float):
    """`count` directional lights on a Fibonacci sphere (a seeded random
    rotation of it) with weights from a synthetic sky: w proportional to
    0.2 + max(0, d_z)^2 (a bright zenith), normalised to sum to 1. Stands in
    for the directions and weights sampled from an environment map."""
    rng = np.random.default_rng(seed)
    i = np.arange(count) + 0.5
    z = 1 - 2 * i / count
    phi = np.pi * (1 + 5 ** 0.5) * i
    r = np.sqrt(1 - z * z)
    dirs = np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w_, x, y, zq = q
    R = np.array([[1 - 2 * (y * y + zq * zq), 2 * (x * y - w_ * zq), 2 * (x * zq + w_ * y)],
                  [2 * (x * y + w_ * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w_ * x)],
                  [2 * (x * zq - w_ * y), 2 * (y * zq + w_ * x), 1 - 2 * (x * x + y * y)]])
    dirs = dirs @ R.T
    w = 0.2 + np.maximum(dirs[:, 2], 0.0) ** 2
    w = w / w.sum()
    return [make_directional(d, width, height, ortho_width) for d in dirs], w


def random_views(count: int, seed: int, radius: float, width: int, height: int,
                 fov_deg: float) -> List[View]:
    """``count`` views on the sphere of ``radius`` looking at the origin."""
    rng = np.random.default_rng(seed)
    return [make_view(rng.standard_normal(3), radius, width, height, fov_deg)
            for _ in range(count)]


def scene_small(seed: int = 0):
    """4,096 Gaussians in [-1,1]^3, 4 lobes, MLPs off; 128^2 camera (40 deg)
    and 128^2 light splat (60 deg), both at radius 4."""
    sc = make_scene(4096, 4, seed, means="cube")
    rng = np.random.default_rng(1)
    cam = make_view(rng.standard_normal(3), 4.0, 128, 128, 40.0)
    light = make_view(rng.standard_normal(3), 4.0, 128, 128, 60.0)
    return sc, cam, light


def scene_full(seed: int = 0, n: int = 300_000):
    """300K Gaussians on a shell of radius U[0.8,1], 8 lobes, both MLPs on;
    800^2 camera and 1024^2 light splat, both 40 deg at radius 4."""
    sc = make_scene(n, 8, seed, means="shell", mlps=True)
    rng = np.random.default_rng(1)
    cam = make_view(rng.standard_normal(3), 4.0, 800, 800, 40.0)
    light = make_view(rng.standard_normal(3), 4.0, 1024, 1024, 40.0)
    return sc, cam, light


def scene_fluffy(seed: int = 0, n: int = 1_500_000):
    """1.5M Gaussians: 70 % fluffy volume, 30 % shell as in ``scene_full``."""
    return make_scene(n, 8, seed, means="shell", mlps=True, fluffy_fraction=0.7)


def fluffy_pairs(count: int, seed: int = 6):
    """(camera, light) pairs of the dense scene's training step: camera
    1024^2 at 40 deg and light splat 2048^2 at 60 deg, both at radius 4 in
    uniformly random directions."""
    rng = np.random.default_rng(seed)
    return [(make_view(rng.standard_normal(3), 4.0, 1024, 1024, 40.0),
             make_view(rng.standard_normal(3), 4.0, 2048, 2048, 60.0)) for _ in range(count)]


def scene_gradcheck(seed: int = 0, n: int = 256, k: int = 4, mlps: bool = True):
    """Small scene for gradient checks: log-scales N(-2, 0.3) so that splats
    cover several pixels of a 32^2 image."""
    sc = make_scene(n, k, seed, means="cube", log_scale_mu=(-2.0, -2.0, -2.0),
                    log_scale_sd=(0.3, 0.3, 0.3), mlps=mlps)
    rng = np.random.default_rng(1)
    cam = make_view(rng.standard_normal(3), 4.0, 32, 32, 40.0)
    light = make_view(rng.standard_normal(3), 4.0, 32, 32, 60.0)
    return sc, cam, light


def concat_scenes(a: Scene, b: Scene) -> Scene:
    """The Gaussians of a, then those of b (a's MLPs)."""
    cat = lambda x, y, ax: np.ascontiguousarray(np.concatenate([x, y], ax))  # noqa: E731
    return Scene(mean=cat(a.mean, b.mean, 1), log_scale=cat(a.log_scale, b.log_scale, 1),
                 rot=cat(a.rot, b.rot, 1), opacity_logit=cat(a.opacity_logit, b.opacity_logit, 0),
                 shade_rot=cat(a.shade_rot, b.shade_rot, 1), albedo=cat(a.albedo, b.albedo, 1),
                 lobe_axis=cat(a.lobe_axis, b.lobe_axis, 2), lobe_log_sharp=cat(a.lobe_log_sharp, b.lobe_log_sharp, 1),
                 lobe_amp=cat(a.lobe_amp, b.lobe_amp, 2), feat=cat(a.feat, b.feat, 1), phi=a.phi, psi=a.psi,
                 basis=None if a.basis is None else dataclasses.replace(
                     a.basis, spec_albedo=cat(a.basis.spec_albedo, b.basis.spec_albedo, 1),
                     weight=cat(a.basis.weight, b.basis.weight, 1), latent=cat(a.basis.latent, b.basis.latent, 1)))


def scene_needles(seed: int = 0, n_needles: int = 60, n_blobs: int = 340, mlps: bool = True):
    """Long thin needles (log-scales N(-1.2, 0.2), N(-4.5, 0.3), N(-4.5, 0.3)
    in [-1,1]^3) among small blobs (log-scales N(-3, 0.3)): in a 256^2 light
    view at 60 deg many needles span 16 tiles or more with a bounding box
    several times their ellipse (the banded shadow-denominator path).
    Camera 128^2 at 40 deg; both views at radius 4."""
    nd = make_scene(n_needles, 4, seed, means="cube", log_scale_mu=(-1.2, -4.5, -4.5),
                    log_scale_sd=(0.2, 0.3, 0.3), mlps=mlps)
    bl = make_scene(n_blobs, 4, seed + 1000, means="cube", log_scale_mu=(-3.0, -3.0, -3.0),
                    log_scale_sd=(0.3, 0.3, 0.3))
    rng = np.random.default_rng(seed + 1)
    cam = make_view(rng.standard_normal(3), 4.0, 128, 128, 40.0)
    light = make_view(rng.standard_normal(3), 4.0, 256, 256, 60.0)
    return concat_scenes(nd, bl), cam, light


def perturb_scene(sc: Scene, seed: int, mean_sd: float = 0.01,
                  colour_sd: float = 0.05) -> Scene:
    """Target scene for the training step: means + N(0, mean_sd), albedo and
    lobe amplitudes (or the basis scene's specular albedo) + N(0, colour_sd),
    unclamped; everything else shared."""
    rng = np.random.default_rng(seed)
    f = np.float32
    out = dataclasses.replace(sc)
    out.mean = (sc.mean.astype(np.float64) + rng.normal(0, mean_sd, sc.mean.shape)).astype(f)
    out.albedo = (sc.albedo.astype(np.float64) + rng.normal(0, colour_sd, sc.albedo.shape)).astype(f)
    out.lobe_amp = (sc.lobe_amp.astype(np.float64) + rng.normal(0, colour_sd, sc.lobe_amp.shape)).astype(f)
    if sc.basis is not None:     # the specular albedo of the shared-basis appearance
        sp = sc.basis.spec_albedo
        out.basis = dataclasses.replace(
            sc.basis, spec_albedo=(sp.astype(np.float64) + rng.normal(0, colour_sd, sp.shape)).astype(f))
    return out


def subset(sc: Scene, idx) -> Scene:
    """Scene restricted to Gaussians ``idx`` (MLPs shared)."""
    idx = np.asarray(idx)
    return Scene(
        mean=np.ascontiguousarray(sc.mean[:, idx]),
        log_scale=np.ascontiguousarray(sc.log_scale[:, idx]),
        rot=np.ascontiguousarray(sc.rot[:, idx]),
        opacity_logit=np.ascontiguousarray(sc.opacity_logit[idx]),
        shade_rot=np.ascontiguousarray(sc.shade_rot[:, idx]),
        albedo=np.ascontiguousarray(sc.albedo[:, idx]),
        lobe_axis=np.ascontiguousarray(sc.lobe_axis[:, :, idx]),
        lobe_log_sharp=np.ascontiguousarray(sc.lobe_log_sharp[:, idx]),
        lobe_amp=np.ascontiguousarray(sc.lobe_amp[:, :, idx]),
        feat=np.ascontiguousarray(sc.feat[:, idx]),
        phi=sc.phi, psi=sc.psi,
        basis=None if sc.basis is None else dataclasses.replace(
            sc.basis, spec_albedo=np.ascontiguousarray(sc.basis.spec_albedo[:, idx]),
            weight=np.ascontiguousarray(sc.basis.weight[:, idx]),
            latent=np.ascontiguousarray(sc.basis.latent[:, idx])),
    )


def make_basis_scene(n: int, seed: int = 0, k: int = 8, mlps: bool = True, **geometry) -> Scene:
    """A scene with the paper's appearance model (Sec. 4.1 shared basis of
    `k` anisotropic angular Gaussians; Sec. 4.2 / 4.3 MLP form).

    Geometry, opacity, rho_d and shading frames are drawn exactly as
    ``make_scene(n, 0, seed, mlps=False, **geometry)`` draws them (no
    per-Gaussian lobes). A second generator, seeded with (seed, 7), then
    draws in this order: rho_s U[0,1]^3, weights alpha U[0,1]^k, latent
    N(0, 0.1)^6 per Gaussian; per basis a random unit frame quaternion,
    sigma_x and sigma_y U[0.3, 1.0] (anisotropic; the paper initialises
    0.5 and 1.0) and sigma_z U[0.13, 0.69] (the paper's initial range),
    stored as logs; then, when `mlps`, Phi 61 -> 32 -> 32 -> 32 -> 1 and Psi
    60 -> 128 -> 128 -> 128 -> 3 (Xavier-uniform weights, zero biases, layer
    order)."""
    sc = make_scene(n, 0, seed, mlps=False, **geometry)
    rng = np.random.default_rng([seed, 7])
    f = np.float32
    spec = rng.uniform(0.0, 1.0, size=(n, 3))
    weight = rng.uniform(0.0, 1.0, size=(n, k))
    latent = rng.normal(0.0, 0.1, size=(n, LATENT_DIM))
    brot = _unit_rows(rng.standard_normal((k, 4)))
    sxy = rng.uniform(0.3, 1.0, size=(k, 2))
    sz = rng.uniform(0.13, 0.69, size=(k, 1))
    log_sigma = np.log(np.concatenate([sxy, sz], 1))
    sc.basis = BasisAppearance(
        spec_albedo=np.ascontiguousarray(spec.T, f),
        weight=np.ascontiguousarray(weight.T, f),
        latent=np.ascontiguousarray(latent.T, f),
        basis_rot=np.ascontiguousarray(brot, f),
        basis_log_sigma=np.ascontiguousarray(log_sigma, f),
    )
    if mlps:
        sc.phi = _make_mlp(rng, PHI_BASIS_IN, 1, hidden=PHI_BASIS_HIDDEN)
        sc.psi = _make_mlp(rng, PSI_BASIS_IN, 3, hidden=PSI_BASIS_HIDDEN)
    return sc


def scene_basis_small(seed: int = 0, n: int = 4096, mlps: bool = True):
    """``scene_small``'s geometry and views with the paper's appearance."""
    sc = make_basis_scene(n, seed, means="cube", mlps=mlps)
    _, cam, light = scene_small(seed)
    return sc, cam, light


def scene_basis_full(seed: int = 0, n: int = 300_000):
    """``scene_full``'s geometry and views (300K shell Gaussians, 800^2
    camera, 1024^2 light) with the paper's appearance and MLPs."""
    sc = make_basis_scene(n, seed, means="shell", mlps=True)
    rng = np.random.default_rng(1)
    cam = make_view(rng.standard_normal(3), 4.0, 800, 800, 40.0)
    light = make_view(rng.standard_normal(3), 4.0, 1024, 1024, 40.0)
    return sc, cam, light


def scene_basis_gradcheck(seed: int = 0, n: int = 256, mlps: bool = True):
    """``scene_gradcheck``'s geometry and views with the paper's appearance."""
    sc = make_basis_scene(n, seed, means="cube", log_scale_mu=(-2.0, -2.0, -2.0),
                          log_scale_sd=(0.3, 0.3, 0.3), mlps=mlps)
    _, cam, light = scene_gradcheck(seed, n=8, k=1, mlps=False)
    return sc, cam, light
