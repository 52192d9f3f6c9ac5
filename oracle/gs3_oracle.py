"""FP64 reference of GS^3's triple splatting (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may use this module. It is a plain, slow, brute-force statement of what the
path computes: every pixel gathers every Gaussian whose 2D footprint can
reach it, sorts them, and composites them front to back, with no tiles,
blocking or fusion. Inputs are plain arrays (numpy or torch) of raw scene
parameters; everything is evaluated in torch float64 on the CPU, so torch
autograd of ``render`` gives reference gradients.

Paper sections followed:
  Sec. 3, Eq. 1      spatial Gaussian, covariance R S S^T R^T
  Sec. 3, Eq. 2-3    projected splats, sort, front-to-back blend
  Sec. 4, Fig. 2     deferred pipeline: final = shading * shadow + residual
  Sec. 4.1, Eq. 4-7  reflectance: modified Lambertian + angular Gaussians
  Sec. 4.2, Fig. 3   shadow splatting, beta-weighted averaging, 0.015 bias
  Sec. 4.2, Eq. 8    shadow refinement MLP Phi
  Sec. 4.3           residual RGB MLP Psi

Readings of points the paper leaves open (camera model, EWA constants,
cut-offs, sort keys, bias semantics) are the named constants of ``Consts``
and the conventions stated in each function's docstring.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import Dict, Optional, Sequence

import numpy as np
import torch

__all__ = [
    "Consts", "SMOOTH", "DT", "ELU_ALPHA", "EPS_D",
    "as_t", "scene_tensors", "quat_to_rotmat", "covariance", "look_at",
    "focal", "project", "tile_rects", "bin_tiles", "pixel_entries",
    "shadow_pass", "shadow_accumulate", "shadow_values", "splat_extent", "diffuse", "angular_gaussian",
    "lobe_frame", "shade", "mlp_forward", "camera_pass", "render",
    "render_images", "sigmoid", "l1_loss", "hit_threshold", "hit_margin", "transmittance_relerr",
    "AMB_BUDGET", "HIT_KAPPA", "pair_key", "ssim_window", "ssim_map", "dssim_loss", "adam_step",
    "SSIM_C1", "SSIM_C2", "SSIM_WINDOW", "SSIM_SIGMA", "LOSS_LAMBDA", "CANDIDATE_CUT", "is_ortho",
    "render_env", "PE_BANDS", "LEAKY_SLOPE", "positional_encoding", "shade_basis", "basis_mlp_inputs",
]

DT = torch.float64

# Sec. 4.1, Eq. 5: the ELU hyper-parameter and epsilon are both 0.01.
ELU_ALPHA = 0.01
EPS_D = 0.01

# Sec. 4.2 / 4.3 (the paper's MLP form): 4-band positional encoding of the
# centre and the light / view direction, leaky ReLU after each hidden layer.
# The paper gives neither the encoding's frequencies nor the slope; the
# readings are frequencies 2^k pi (k = 0..3) with the input itself kept, and
# the customary slope 0.01.
PE_BANDS = 4
LEAKY_SLOPE = 0.01


@dataclass(frozen=True)
class Consts:
    """Rasteriser conventions the paper inherits from vanilla Gaussian
    splatting without stating them (Sec. 3), plus the paper's shadow bias.

    near        cull a Gaussian whose view-space z is <= near
    clamp_frac  clamp x/z and y/z to +-clamp_frac*tan(half fov) in the
                Jacobian only (EWA)
    dilation    added to both diagonal entries of the 2D covariance (px^2)
    cutoff      a pixel is hit only if power >= -cutoff (3-sigma ellipse)
    alpha_min   ... and alpha >= alpha_min
    alpha_max   alpha = min(alpha_max, opacity * exp(power))
    t_min       camera pass stops before a hit that would take T below t_min
    shadow_bias Sec. 4.2: k shadows j only if dist_k < dist_j - bias
    """
    near: float = 0.2
    clamp_frac: float = 1.3
    dilation: float = 0.3
    cutoff: float = 4.5
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    shadow_bias: float = 0.015


# Smooth mode for finite-difference gradient checks: no thresholds anywhere,
# every Gaussian reaches every pixel, no clamp, no early stop, no dilation.
SMOOTH = Consts(dilation=0.0, cutoff=math.inf, alpha_min=0.0, alpha_max=1.0,
                t_min=0.0, shadow_bias=0.0)


def as_t(x) -> torch.Tensor:
    """float64 CPU tensor view of an array (keeps autograd if already one)."""
    if isinstance(x, torch.Tensor):
        return x if x.dtype == DT else x.to(DT)
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


def sigmoid(x):
    return 1.0 / (1.0 + torch.exp(-x))


def scene_tensors(scene, requires_grad: bool = False) -> Dict[str, torch.Tensor]:
    """Raw per-Gaussian parameters as float64 tensors, Gaussian index first.

    ``scene`` has attributes mean [3,N], log_scale [3,N], rot [4,N],
    opacity_logit [N], shade_rot [4,N], albedo [3,N], lobe_axis [K,3,N],
    lobe_log_sharp [K,N], lobe_amp [K,3,N], feat [F,N]."""
    def t(a, perm=None):
        x = as_t(a).clone()
        if perm is not None:
            x = x.permute(*perm).contiguous()
        return x.requires_grad_(requires_grad)
    return {
        "mean": t(scene.mean, (1, 0)),
        "log_scale": t(scene.log_scale, (1, 0)),
        "rot": t(scene.rot, (1, 0)),
        "opacity_logit": t(scene.opacity_logit),
        "shade_rot": t(scene.shade_rot, (1, 0)),
        "albedo": t(scene.albedo, (1, 0)),
        "lobe_axis": t(scene.lobe_axis, (2, 0, 1)),      # [N,K,3]
        "lobe_log_sharp": t(scene.lobe_log_sharp, (1, 0)),  # [N,K]
        "lobe_amp": t(scene.lobe_amp, (2, 0, 1)),        # [N,K,3]
        "feat": t(scene.feat, (1, 0)),
        **_basis_tensors(scene, t),
    }


def _basis_tensors(scene, t) -> Dict[str, torch.Tensor]:
    """The shared-basis appearance of Sec. 4.1 when the scene carries one
    (``scene.basis``): per Gaussian rho_s [N,3], the basis weights alpha
    [N,K] and the latent l [N,6]; shared by all Gaussians, each basis angular
    Gaussian's frame quaternion [K,4] and log(sigma_x, sigma_y, sigma_z)
    [K,3]."""
    b = getattr(scene, "basis", None)
    if b is None:
        return {}
    return {
        "spec_albedo": t(b.spec_albedo, (1, 0)),
        "basis_weight": t(b.weight, (1, 0)),
        "latent": t(b.latent, (1, 0)),
        "basis_rot": t(b.basis_rot),
        "basis_log_sigma": t(b.basis_log_sigma),
    }


# ---------------------------------------------------------------- geometry

def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of quaternion q = (w, x, y, z) after normalising it.
    Used for R in Eq. 1 and for the world-to-shading rotation of Sec. 4.1."""
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    rows = [
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ]
    return torch.stack(rows, -1).reshape(q.shape[:-1] + (3, 3))


def covariance(log_scale: torch.Tensor, rot: torch.Tensor) -> torch.Tensor:
    """Sec. 3, Eq. 1: Sigma = R S S^T R^T with S = diag(exp(log_scale))."""
    R = quat_to_rotmat(rot)
    M = R * torch.exp(log_scale)[..., None, :]   # R @ diag(s)
    return M @ M.transpose(-1, -2)


def look_at(eye, target) -> torch.Tensor:
    """World-to-camera rotation (rows: right, down, forward).

    Camera axes x right, y down, z forward; world up is +z unless the view
    direction is within acos(0.99) of it, then +y."""
    eye, target = as_t(eye), as_t(target)
    f = target - eye
    f = f / torch.linalg.norm(f)
    up = as_t([0.0, 0.0, 1.0]) if abs(float(f[2])) <= 0.99 else as_t([0.0, 1.0, 0.0])
    r = torch.linalg.cross(f, up)
    r = r / torch.linalg.norm(r)
    d = torch.linalg.cross(f, r)
    return torch.stack([r, d, f])


def focal(view) -> float:
    """Focal length in pixels from the horizontal field of view."""
    return (view.width / 2.0) / math.tan(view.fov / 2.0)


def is_ortho(view) -> bool:
    """An orthographic view (a directional light, Sec. 4.5)."""
    return getattr(view, "projection", "perspective") == "orthographic"


def project(mean: torch.Tensor, cov: torch.Tensor, view, consts: Consts,
            depth_mode: str) -> Dict[str, torch.Tensor]:
    """Project 3D Gaussians to 2D splats (Sec. 3; EWA splatting as in GS).

    t = R_v (mu - eye); cull t_z <= near. Jacobian of the pinhole map at t
    with x/z, y/z clamped to +-clamp_frac*tan(half fov); Sigma' = J R_v Sigma
    R_v^T J^T + dilation*I; cull det <= 0; conic = Sigma'^-1; centre
    (f t_x/t_z + W/2, f t_y/t_z + H/2). The depth key is t_z for the camera
    ("z") and |mu - eye| toward the light ("dist", Sec. 4.2).

    An orthographic view (a directional light: Sec. 4.5 switches the shadow
    splat to an orthographic projection) maps t to (s t_x + W/2, s t_y +
    H/2) with s = W / ortho_width pixels per world unit, so J = [[s, 0, 0],
    [0, s, 0]]; its distance key is t_z, the depth along the light
    direction."""
    W, H = view.width, view.height
    Rv = look_at(view.eye, view.target)
    eye = as_t(view.eye)
    t = (mean - eye) @ Rv.T
    tz = t[:, 2]
    valid = tz > consts.near
    tzs = torch.where(valid, tz, torch.ones_like(tz))
    zero = torch.zeros_like(tz)
    ortho = is_ortho(view)
    if ortho:
        f = W / view.ortho_width
        sv = torch.full_like(tz, f)
        J = torch.stack([torch.stack([sv, zero, zero], -1), torch.stack([zero, sv, zero], -1)], 1)
    else:
        f = focal(view)
        lim_x = consts.clamp_frac * (W / 2.0) / f
        lim_y = consts.clamp_frac * (H / 2.0) / f
        xr = torch.clamp(t[:, 0] / tzs, -lim_x, lim_x)
        yr = torch.clamp(t[:, 1] / tzs, -lim_y, lim_y)
        J = torch.stack([
            torch.stack([f / tzs, zero, -f * xr / tzs], -1),
            torch.stack([zero, f / tzs, -f * yr / tzs], -1)], 1)        # [N,2,3]
    cov_cam = Rv @ cov @ Rv.T
    cov2 = J @ cov_cam @ J.transpose(1, 2)
    a = cov2[:, 0, 0] + consts.dilation
    b = cov2[:, 0, 1]
    c = cov2[:, 1, 1] + consts.dilation
    det = a * c - b * b
    valid = valid & (det > 0)
    dets = torch.where(valid, det, torch.ones_like(det))
    conic = torch.stack([c / dets, -b / dets, a / dets], -1)
    if ortho:
        u = f * t[:, 0] + W / 2.0
        v = f * t[:, 1] + H / 2.0
    else:
        u = f * t[:, 0] / tzs + W / 2.0
        v = f * t[:, 1] / tzs + H / 2.0
    if depth_mode == "z" or (depth_mode == "dist" and ortho):
        depth = tz
    elif depth_mode == "dist":
        depth = torch.linalg.norm(mean - eye, dim=-1)
    else:
        raise ValueError(depth_mode)
    return {"u": u, "v": v, "cov2": torch.stack([a, b, c], -1), "conic": conic,
            "depth": depth, "valid": valid, "tz": tz, "det": det}


# ----------------------------------------------------------------- binning

def splat_extent(proj, opacity: torch.Tensor, consts: Consts):
    """Integer pixel extent of each splat's hit region, used for binning.

    A pixel is hit only where power >= -cutoff and opacity * exp(power) >=
    alpha_min, i.e. where power >= -p with p = min(cutoff, ln(opacity /
    alpha_min)): an ellipse whose bounding box has half-widths
    sqrt(2 p Sigma'_xx), sqrt(2 p Sigma'_yy). Returns (ix, iy, rx, ry) int64
    arrays: ix = floor(u), iy = floor(v), rx/ry the half-widths rounded up;
    rx = ry = -1 for culled splats (behind the near plane, degenerate, or
    never reaching alpha_min)."""
    with torch.no_grad():
        op = opacity.detach()
        p = torch.full_like(op, consts.cutoff)
        if consts.alpha_min > 0:
            p = torch.minimum(p, torch.log(op / consts.alpha_min))
        ok = proj["valid"] & (p > 0)
        big = float(1 << 20)
        a = proj["cov2"][:, 0].detach().clamp_min(0)
        c = proj["cov2"][:, 2].detach().clamp_min(0)
        rx = torch.ceil(torch.sqrt(2 * p.clamp_min(0) * a)).clamp_max(big)
        ry = torch.ceil(torch.sqrt(2 * p.clamp_min(0) * c)).clamp_max(big)
        lim = float(1 << 30)
        ix = torch.floor(proj["u"].detach().clamp(-lim, lim))
        iy = torch.floor(proj["v"].detach().clamp(-lim, lim))
        rx = torch.where(ok, rx, torch.full_like(rx, -1))
        ry = torch.where(ok, ry, torch.full_like(ry, -1))
    return (ix.numpy().astype(np.int64), iy.numpy().astype(np.int64),
            rx.numpy().astype(np.int64), ry.numpy().astype(np.int64))


def tile_rects(ix, iy, rx, ry, W: int, H: int, tile: int = 16):
    """Tiles a splat is binned to: the 16x16 tiles covering pixel columns
    ix-rx .. ix+rx and rows iy-ry .. iy+ry, clamped to the grid; empty when
    rx <= 0 or ry <= 0 or the rectangle misses the image."""
    tx = (W + tile - 1) // tile
    ty = (H + tile - 1) // tile
    ix, iy = np.asarray(ix, np.int64), np.asarray(iy, np.int64)
    rx, ry = np.asarray(rx, np.int64), np.asarray(ry, np.int64)
    x0 = np.maximum((ix - rx) // tile, 0)
    x1 = np.minimum((ix + rx) // tile, tx - 1)
    y0 = np.maximum((iy - ry) // tile, 0)
    y1 = np.minimum((iy + ry) // tile, ty - 1)
    empty = (x0 > x1) | (y0 > y1) | (rx <= 0) | (ry <= 0)
    return x0, x1, y0, y1, empty


def bin_tiles(ix, iy, rx, ry, depth, W: int, H: int, tile: int = 16):
    """Brute-force binning (Sec. 3 "sorted"; Sec. 4.2 sorted by distance).

    For every tile, the ids of the splats whose rect covers it, ordered by
    (float32 depth bits, id). Returns (counts [tiles], flat id list, keys
    [P] uint64 = tile << 32 | depth bits) laid out tile by tile, exactly as a
    sort of (tile, depth, id) would. Inputs: integer extents (see
    ``splat_extent``) and float32 depths (>= 0)."""
    depth = np.asarray(depth, np.float32)
    x0, x1, y0, y1, empty = tile_rects(ix, iy, rx, ry, W, H, tile)
    tx = (W + tile - 1) // tile
    ty = (H + tile - 1) // tile
    dbits = depth.view(np.uint32).astype(np.uint64)
    counts = np.zeros(tx * ty, np.int64)
    lists, keys = [], []
    ids = np.arange(depth.shape[0])
    for t_id in range(tx * ty):
        gx, gy = t_id % tx, t_id // tx
        sel = (~empty) & (x0 <= gx) & (gx <= x1) & (y0 <= gy) & (gy <= y1)
        members = ids[sel]
        members = members[np.lexsort((members, dbits[members]))]   # by depth bits, then id
        counts[t_id] = members.size
        lists.append(members)
        keys.append((np.uint64(t_id) << np.uint64(32)) | dbits[members])
    return counts, np.concatenate(lists), np.concatenate(keys)


# -------------------------------------------------------- per-pixel entries

# Error model of a float32 evaluation, used only to flag outputs whose value
# hangs on a threshold decision (cut-off, alpha minimum, early stop) that a
# float32 evaluation may take differently from this float64 one. (Depth
# order and the shadow-bias test are decided on float32 keys in float32
# arithmetic on both sides, so they need no flag.)
#
# The float32 evaluation it describes: splat centre, conic and opacity
# rounded once to float32 from an exact value; the pixel offset d formed
# relative to an origin within 16 px of the pixel (a tile corner); the
# quadratic power = -(a dx^2 + 2 b dx dy + c dy^2) / 2 and the threshold
# p = min(cutoff, ln(opacity / alpha_min)) each evaluated in a handful of
# float32 operations. With u = 2^-24 (float32 unit roundoff):
#   - each conic coefficient carries 2 roundings and each quadratic term up
#     to 5 more: at most 3.5 u S, S = |a| dx^2 + 2 |b dx dy| + |c| dy^2
#     (S, not |power|: the terms can cancel for elongated splats);
#   - the offset error is at most u (2 |d| + 17) per axis (the centre's
#     fractional part, the offset from the origin, the difference), times
#     the gradient |conic d| of the power;
#   - the threshold: the opacity ratio, a logarithm within 2 ulp and the
#     scaling, at most u (4 + 6 p).
# HIT_KAPPA widens the sum by half. A float32 simulation of this evaluation
# (three operation orders, 10^7 pairs near the threshold, elongated splats
# included) found every decision flip inside the margin and the largest
# error at 0.73 of the unwidened sum (tests/test_oracle_pins.py).
_U32 = 2.0 ** -24
HIT_KAPPA = 1.5
AMB_BUDGET = 5e-5        # an output is ambiguous when it could move this much


def CANDIDATE_CUT(cutoff: float) -> float:
    """Power threshold of the (pixel, splat) pairs the oracle considers:
    1 % beyond the cut-off, far wider than the float32 error margin."""
    return cutoff * (1 + 1e-2) + 1e-2


def hit_threshold(opacity: torch.Tensor, consts: Consts) -> torch.Tensor:
    """p with hit <=> power >= -p: min(cutoff, ln(opacity / alpha_min))
    (the cut-off and the alpha >= alpha_min test of Sec. 3 in one bound)."""
    p = torch.full_like(opacity, consts.cutoff)
    if consts.alpha_min > 0:
        p = torch.minimum(p, torch.log(opacity / consts.alpha_min))
    return p


def hit_margin(dx, dy, ca, cb, cc, p) -> torch.Tensor:
    """Bound on how far a float32 evaluation of power + p can fall from the
    exact value for pixel offset (dx, dy), conic (ca, cb, cc) and threshold
    p (see the error model above); a pair whose |power + p| is within it is
    a hit or a miss depending on rounding."""
    S = ca.abs() * dx * dx + 2 * (cb * dx * dy).abs() + cc.abs() * dy * dy
    gx = (ca * dx + cb * dy).abs()
    gy = (cb * dx + cc * dy).abs()
    pos = gx * (2 * dx.abs() + 17.0) + gy * (2 * dy.abs() + 17.0)
    return HIT_KAPPA * _U32 * (3.5 * S + pos + 4.0 + 6.0 * p.abs())


def transmittance_relerr(alpha_full, hit, margin, consts: Consts) -> torch.Tensor:
    """Per hit, a bound on the relative float32 error of its factor
    (1 - alpha) in a transmittance product, plus the product's own
    rounding: alpha = min(alpha_max, opacity exp(power)) carries the power
    error (margin) and a few roundings (exp, the opacity, the product),
    which (1 - alpha) amplifies by alpha / (1 - alpha); a clamped alpha is
    exact up to the float32 rounding of alpha_max."""
    am32 = float(np.float32(consts.alpha_max))
    clamped = alpha_full >= consts.alpha_max
    one_m = (1.0 - alpha_full).clamp_min(1e-30)
    r_free = alpha_full * (margin / HIT_KAPPA + 4 * _U32) / one_m
    r_clamp = abs(am32 - consts.alpha_max) / one_m
    r = torch.where(clamped, r_clamp, r_free) + 3 * _U32
    return torch.where(hit, HIT_KAPPA * r, torch.zeros_like(r))


def pair_key(gid, px, py, W: int, H: int):
    """Integer name of the pair (Gaussian gid, pixel (px, py)) of a W x H
    view: gid * W * H + py * W + px."""
    return gid * (W * H) + py * W + px


def pixel_entries(proj, W: int, H: int, opacity: torch.Tensor, consts: Consts,
                  pixels: Optional[torch.Tensor] = None, rows=None, flips=None):
    """Every (pixel, Gaussian) pair whose power can reach the cut-off,
    grouped per pixel and sorted by (depth, id): a padded [P, L] layout.

    The hit test (Sec. 3, Eq. 2): d = pixel centre (i+0.5, j+0.5) - centre,
    power = -1/2 d^T conic d, alpha = min(alpha_max, opacity * exp(power)),
    beta = exp(power) (the splat's density at the pixel centre); a hit needs
    power >= -cutoff and alpha >= alpha_min. Pairs just outside the cut-off
    are kept as non-hits so that threshold ambiguity can be measured.

    ``rows`` = (y0, y1) selects a band of full rows, else ``pixels`` is a
    1-D tensor of flat pixel indices (y*W + x); default all pixels.

    ``flips`` (optional 1-D int64 tensor of pair keys, see ``pair_key``)
    inverts the hit decision of those pairs. It is meant for pairs the
    error model flags: their decision is a rounding matter, so a float32
    evaluation may take it either way, and a comparison supplies the
    decision it observed."""
    u, v, conic, cov2, depth, valid = (proj["u"], proj["v"], proj["conic"],
                                       proj["cov2"], proj["depth"], proj["valid"])
    n = u.shape[0]
    if rows is not None:
        ylo, yhi = rows
        xlo, xhi = 0, W
        pix_set = None
    else:
        if pixels is None:
            pixels = torch.arange(W * H)
        pixels = torch.as_tensor(pixels, dtype=torch.int64)
        assert torch.unique(pixels).numel() == pixels.numel(), "pixels must be distinct"
        py_all, px_all = pixels // W, pixels % W
        ylo, yhi = int(py_all.min()), int(py_all.max()) + 1
        xlo, xhi = int(px_all.min()), int(px_all.max()) + 1
        pix_set = torch.full(((yhi - ylo) * (xhi - xlo),), -1, dtype=torch.int64)
        pix_set[(py_all - ylo) * (xhi - xlo) + (px_all - xlo)] = torch.arange(pixels.numel())
    with torch.no_grad():
        # candidates: the pixels of the ellipse power >= -cut, found through
        # its bounding box (half-widths sqrt(2 cut Sigma'_xx), sqrt(2 cut
        # Sigma'_yy)); the cut is 1 % beyond the cut-off so that near misses
        # within the float32 error margin are seen. Pairs outside that
        # ellipse can neither hit nor be flagged and are dropped.
        cut = CANDIDATE_CUT(consts.cutoff)
        uu, vv = u.detach(), v.detach()
        if math.isinf(cut):
            cx0 = torch.full((n,), xlo, dtype=torch.int64)
            cx1 = torch.full((n,), xhi - 1, dtype=torch.int64)
            cy0 = torch.full((n,), ylo, dtype=torch.int64)
            cy1 = torch.full((n,), yhi - 1, dtype=torch.int64)
        else:
            hx = torch.sqrt(2 * cut * cov2[:, 0].detach().clamp_min(0))
            hy = torch.sqrt(2 * cut * cov2[:, 2].detach().clamp_min(0))
            big = 2.0 ** 40
            cx0 = torch.ceil((uu - hx - 0.5).clamp(-big, big)).to(torch.int64).clamp(xlo, xhi)
            cx1 = torch.floor((uu + hx - 0.5).clamp(-big, big)).to(torch.int64).clamp(xlo - 1, xhi - 1)
            cy0 = torch.ceil((vv - hy - 0.5).clamp(-big, big)).to(torch.int64).clamp(ylo, yhi)
            cy1 = torch.floor((vv + hy - 0.5).clamp(-big, big)).to(torch.int64).clamp(ylo - 1, yhi - 1)
        nx = (cx1 - cx0 + 1).clamp_min(0)
        ny = (cy1 - cy0 + 1).clamp_min(0)
        cnt = torch.where(valid, nx * ny, torch.zeros_like(nx))
        gid = torch.repeat_interleave(torch.arange(n), cnt)
        start = torch.cumsum(cnt, 0) - cnt
        local = torch.arange(gid.numel()) - start[gid]
        px = cx0[gid] + local % nx[gid]
        py = cy0[gid] + local // nx[gid]
        if pix_set is None:
            pidx = (py - ylo) * W + px
            n_pix = (yhi - ylo) * W
        else:
            pidx = pix_set[(py - ylo) * (xhi - xlo) + (px - xlo)]
            keep = pidx >= 0
            gid, px, py, pidx = gid[keep], px[keep], py[keep], pidx[keep]
            n_pix = pixels.numel()
        if not math.isinf(cut):
            ddx = (px.to(DT) + 0.5) - uu[gid]
            ddy = (py.to(DT) + 0.5) - vv[gid]
            cg = conic.detach()[gid]
            pw0 = -0.5 * (cg[:, 0] * ddx * ddx + 2 * cg[:, 1] * ddx * ddy + cg[:, 2] * ddy * ddy)
            keep = pw0 >= -cut
            gid, px, py, pidx = gid[keep], px[keep], py[keep], pidx[keep]
        # sort by (pixel, depth key, id): pairs come in id order, then two
        # stable sorts. The depth key is the depth rounded to float32 (the
        # method's sort key); the order is a discrete decision, so it is
        # taken in the kernel's precision and matches it exactly.
        dep = depth.detach().to(torch.float32).to(DT)[gid]
        o = torch.sort(dep, stable=True).indices
        gid, px, py, pidx, dep = gid[o], px[o], py[o], pidx[o], dep[o]
        o = torch.sort(pidx, stable=True).indices
        gid, px, py, pidx, dep = gid[o], px[o], py[o], pidx[o], dep[o]
        counts = torch.bincount(pidx, minlength=n_pix)
        L = int(counts.max()) if counts.numel() and gid.numel() else 0
        first = torch.cumsum(counts, 0) - counts
        pos = torch.arange(gid.numel()) - first[pidx]
    # differentiable per-pair quantities
    dx = (px.to(DT) + 0.5) - u[gid]
    dy = (py.to(DT) + 0.5) - v[gid]
    ca, cb, cc = conic[gid, 0], conic[gid, 1], conic[gid, 2]
    power = -0.5 * (ca * dx * dx + 2 * cb * dx * dy + cc * dy * dy)
    beta = torch.exp(power)
    alpha_full = torch.clamp(opacity[gid] * beta, max=consts.alpha_max)
    with torch.no_grad():
        hit = (power >= -consts.cutoff) & (alpha_full >= consts.alpha_min)
        key = pair_key(gid, px, py, W, H)
        if flips is not None and len(flips):
            hit = hit ^ torch.isin(key, torch.as_tensor(flips, dtype=torch.int64))
        # threshold ambiguity of this pair (the cut-off or the alpha minimum,
        # both power >= -p): within the float32 error margin of -p
        pw, op = power.detach(), opacity.detach()[gid]
        p_thr = hit_threshold(op, consts)
        fin = torch.isfinite(p_thr)          # no threshold at all without a cut-off and alpha minimum
        p_fin = torch.where(fin, p_thr, torch.zeros_like(p_thr))
        marg = hit_margin(dx.detach(), dy.detach(), ca.detach(), cb.detach(), cc.detach(), p_fin)
        amb = fin & ((pw + p_fin).abs() <= marg)
        t_rel = transmittance_relerr(alpha_full.detach(), hit, marg, consts)

    def pad(x, fill):
        out = torch.full((n_pix, max(L, 1)), fill, dtype=x.dtype)
        return out.index_put((pidx, pos), x)

    return {
        "n_pix": n_pix, "L": L, "gid": gid, "pidx": pidx, "pos": pos,
        "px": px, "py": py, "counts": counts,
        "gid_pad": pad(gid, -1), "hit_pad": pad(hit, False),
        "amb_pad": pad(amb, False),
        "depth_pad": pad(dep, math.inf),
        "alpha_pad": pad(torch.where(hit, alpha_full, torch.zeros_like(alpha_full)), 0.0),
        "alpha_full_pad": pad(alpha_full.detach(), 0.0),
        "beta_pad": pad(torch.where(hit, beta, torch.zeros_like(beta)), 0.0),
        "beta_full_pad": pad(beta.detach(), 0.0),
        "t_relerr_pad": pad(t_rel, 0.0),
        "key_pad": pad(key, -1),
        "marg_pad": pad(marg, 0.0),
    }


def _excl_prefix_product(x: torch.Tensor) -> torch.Tensor:
    """[P, L] -> [P, L+1] with out[:, c] = prod_{k<c} x[:, k] (Eq. 3)."""
    ones = torch.ones(x.shape[0], 1, dtype=x.dtype)
    return torch.cat([ones, torch.cumprod(x, dim=1)], 1)


# ------------------------------------------------------------ shadow pass

def shadow_pass(proj_l, light_view, opacity: torch.Tensor, consts: Consts,
                band_rows: int = 8, pixels=None, flips=None, amb_keys: Optional[list] = None,
                pair_out: Optional[list] = None, den_err: Optional[torch.Tensor] = None):
    """Second splatting (Sec. 4.2, Fig. 3) over the light image.

    Every light pixel m is one shadow ray; its hits are sorted by distance to
    the light. For each hit j the cumulative transmittance in front of it is
    T_m(j) = prod (1 - alpha_km) over hits k on m with
    dist_k < dist_j - shadow_bias (Eq. 3 with the bias of Sec. 4.2; the
    distances are the float32 depth keys and the comparison is evaluated in
    float32, as the kernel does); then num_j += beta_jm T_m(j) and
    den_j += beta_jm. Returns num, den and the
    per-Gaussian ambiguity bound (an upper bound on how far T_j could move
    if float32 took a threshold decision the other way). ``flips`` inverts
    the hit decision of the given pair keys (``pixel_entries``); the keys of
    the pairs the error model flags are appended to ``amb_keys`` when it is
    a list, and every hit's (Gaussian, flat pixel, beta T_m(j), beta) to
    ``pair_out`` when that is a list (its terms of num and den). When
    ``den_err`` (a float64 tensor [n]) is given, each Gaussian's bound on the
    float32 error of its den terms is added to it: beta times the error
    margin of the pair's power (a float32 beta = exp(power) moves by that
    relative amount)."""
    W, H = light_view.width, light_view.height
    n = opacity.shape[0]
    num = torch.zeros(n, dtype=DT)
    den = torch.zeros(n, dtype=DT)
    infl = torch.zeros(n, dtype=DT)
    b = consts.shadow_bias
    if pixels is not None:
        chunks = [("pix", pixels)]
    else:
        chunks = [("rows", (y, min(H, y + band_rows))) for y in range(0, H, band_rows)]
    for kind, arg in chunks:
        e = pixel_entries(proj_l, W, H, opacity, consts,
                          rows=arg if kind == "rows" else None,
                          pixels=arg if kind == "pix" else None, flips=flips)
        if e["L"] == 0:
            continue
        if amb_keys is not None:
            amb_keys.append(e["key_pad"][e["amb_pad"]])
        alpha, beta, dist = e["alpha_pad"], e["beta_pad"], e["depth_pad"]
        hit, gidp = e["hit_pad"], e["gid_pad"]
        prefix = _excl_prefix_product(1.0 - alpha)                  # [P, L+1]
        # occluders: key_k < fl32(key_j - fl32(bias)) -- a discrete decision
        # on float32 keys, evaluated in float32 like the kernel
        thr = (dist.to(torch.float32) - torch.tensor(b, dtype=torch.float32)).to(DT)
        cnt = torch.searchsorted(dist.contiguous(), thr.contiguous(), right=False)
        Tm = torch.gather(prefix, 1, cnt)                           # T_m(j)
        if pair_out is not None:
            kp = e["key_pad"][hit]
            pair_out.append((gidp[hit], kp % (W * H), (beta[hit] * Tm[hit]).detach(), beta[hit].detach()))
        if den_err is not None:
            den_err.index_add_(0, gidp[hit], (beta[hit] * e["marg_pad"][hit]).detach())
        dn, dd = shadow_accumulate(gidp[hit], beta[hit], Tm[hit], n)
        num = num + dn
        den = den + dd
        with torch.no_grad():
            # ambiguity: a threshold flip of j's own pair moves T_j by at most
            # beta_jm / den_j; a threshold flip of an occluder k moves T_m(j)
            # by at most alpha_k times the transmittance in front of k.
            amb = e["amb_pad"]
            af = e["alpha_full_pad"]
            Tk = prefix[:, :-1].detach()
            z1 = torch.zeros(af.shape[0], 1, dtype=DT)
            occ_amb = torch.cat([z1, torch.cumsum(torch.where(amb, af * Tk, torch.zeros_like(af)), 1)], 1)
            occ = torch.gather(occ_amb, 1, cnt)
            bf = e["beta_full_pad"]
            own = torch.where(amb, bf, torch.zeros_like(bf))
            w_all = own + torch.where(hit, bf * occ, torch.zeros_like(bf))
            valid_e = gidp >= 0
            infl = infl.index_add(0, gidp[valid_e], w_all[valid_e])
    return num, den, infl


def shadow_accumulate(gid: torch.Tensor, beta: torch.Tensor, Tm: torch.Tensor, n: int):
    """Sec. 4.2 / Fig. 3: each intersection of Gaussian gid with a shadow ray
    adds beta * T_m to its numerator and beta to its denominator."""
    num = torch.zeros(n, dtype=DT).index_add(0, gid, beta * Tm)
    den = torch.zeros(n, dtype=DT).index_add(0, gid, beta)
    return num, den


def shadow_values(num: torch.Tensor, den: torch.Tensor) -> torch.Tensor:
    """Sec. 4.2: T = sum_m beta_m T_m / sum_m beta_m; 1 where no ray hits."""
    ok = den > 0
    return torch.where(ok, num / torch.where(ok, den, torch.ones_like(den)),
                       torch.ones_like(num))


# ---------------------------------------------------------------- shading

def diffuse(cos_i: torch.Tensor) -> torch.Tensor:
    """Sec. 4.1, Eq. 5: f_d = (ELU(n'.w_i) + eps (1 - 1/e)) / ((1 + eps (1 - 1/e)) pi),
    ELU with alpha = 0.01, eps = 0.01."""
    elu = torch.where(cos_i > 0, cos_i, ELU_ALPHA * (torch.exp(torch.clamp(cos_i, max=0.0)) - 1.0))
    k = EPS_D * (1.0 - math.exp(-1.0))
    return (elu + k) / ((1.0 + k) * math.pi)


def lobe_frame(z: torch.Tensor):
    """An orthonormal [x, y] completing the unit lobe axis z (any completion
    is valid for an isotropic lobe, sigma_x = sigma_y)."""
    helper = torch.where((z[..., 0].abs() < 0.9)[..., None],
                         torch.tensor([1.0, 0.0, 0.0], dtype=DT).expand_as(z),
                         torch.tensor([0.0, 1.0, 0.0], dtype=DT).expand_as(z))
    x = helper - (helper * z).sum(-1, keepdim=True) * z
    x = x / torch.linalg.norm(x, dim=-1, keepdim=True)
    y = torch.linalg.cross(z, x)
    return x, y


def angular_gaussian(h, x, y, z, sx, sy, sz):
    """Sec. 4.1, Eq. 7: G(h') = 1/sigma_z exp(-1/2 (acos(h'.z) *
    sqrt((s'.x/sigma_x)^2 + (s'.y/sigma_y)^2) / sigma_z)^2), with s' the
    normalised projection of h' onto the x-y plane. When that projection
    vanishes (h' = +-z) the anisotropy factor is taken as 1."""
    cz = (h * z).sum(-1)
    theta = torch.arccos(torch.clamp(cz, -1.0, 1.0))
    s = h - cz[..., None] * z
    sn = torch.linalg.norm(s, dim=-1)
    ok = sn > 1e-12
    s = s / torch.where(ok, sn, torch.ones_like(sn))[..., None]
    aniso = torch.sqrt(((s * x).sum(-1) / sx) ** 2 + ((s * y).sum(-1) / sy) ** 2)
    aniso = torch.where(ok, aniso, torch.ones_like(aniso))
    return torch.exp(-0.5 * (theta * aniso / sz) ** 2) / sz


def shade(p: Dict[str, torch.Tensor], light_pos, eye, light_dir=None) -> Dict[str, torch.Tensor]:
    """First splatting (Sec. 4.1, Eq. 4): per-Gaussian colour
    c = rho_d f_d(w_i') + sum_k amp_k G_k(h') in the Gaussian's shading frame.

    w_i, w_o are unit vectors from the centre toward the light and camera;
    w' = R_sh w with R_sh the world-to-shading rotation of the shading
    quaternion; n' = +z. Lobes are isotropic (sigma_x = sigma_y = 1) with
    sigma_z = exp(-log_sharp) and axis normalised in the shading frame;
    amp_k is the lobe's RGB weight (alpha_j rho_s of Eq. 4/6). Unit light
    intensity, no distance fall-off. With ``light_dir`` (a directional
    light, Sec. 4.5) w_i is that unit direction toward the light for every
    Gaussian."""
    mu = p["mean"]
    wi, wo = _directions(mu, light_pos, eye, light_dir)
    Rsh = quat_to_rotmat(p["shade_rot"])
    wi_l = (Rsh @ wi[..., None])[..., 0]
    wo_l = (Rsh @ wo[..., None])[..., 0]
    fd = diffuse(wi_l[:, 2])
    hs = wi_l + wo_l
    hn = torch.linalg.norm(hs, dim=-1, keepdim=True)
    ok = hn > 1e-12
    ez = torch.tensor([0.0, 0.0, 1.0], dtype=DT).expand_as(hs)
    h = torch.where(ok, hs / torch.where(ok, hn, torch.ones_like(hn)), ez)
    z = p["lobe_axis"] / torch.linalg.norm(p["lobe_axis"], dim=-1, keepdim=True)  # [N,K,3]
    x, y = lobe_frame(z)
    sz = torch.exp(-p["lobe_log_sharp"])                       # [N,K]
    G = angular_gaussian(h[:, None, :], x, y, z, 1.0, 1.0, sz)  # [N,K]
    spec = (p["lobe_amp"] * G[..., None]).sum(1)               # [N,3]
    c = p["albedo"] * fd[:, None] + spec
    return {"c": c, "wi": wi, "wo": wo, "fd": fd, "h": h, "G": G}


def _directions(mu, light_pos, eye, light_dir=None):
    """Unit w_i (toward the light, or a directional light's fixed direction)
    and w_o (toward the camera) per Gaussian centre."""
    if light_dir is not None:
        d = as_t(light_dir)
        wi = (d / torch.linalg.norm(d)).expand_as(mu)
    else:
        wi = as_t(light_pos) - mu
        wi = wi / torch.linalg.norm(wi, dim=-1, keepdim=True)
    wo = as_t(eye) - mu
    wo = wo / torch.linalg.norm(wo, dim=-1, keepdim=True)
    return wi, wo


def shade_basis(p: Dict[str, torch.Tensor], light_pos, eye, light_dir=None) -> Dict[str, torch.Tensor]:
    """First splatting with the paper's shared basis (Sec. 4.1, Eq. 4-7 and
    the shared-basis paragraph): c = rho_d f_d(w_i') + rho_s sum_j alpha_j
    G_j(h'), where the K basis angular Gaussians are shared by every spatial
    Gaussian and each spatial Gaussian has its own shading frame, rho_d,
    rho_s (RGB) and weights alpha_j.

    Basis j has a frame [x_j, y_j, z_j] in the shading frame, given by a
    quaternion whose rotation maps shading-frame coordinates to the basis
    frame (the rows of its matrix are x_j, y_j, z_j, the same convention as
    the world-to-shading quaternion), and sigma_x, sigma_y, sigma_z =
    exp(log sigma). G_j is Eq. 7, anisotropic (``angular_gaussian``).
    w_i, w_o, h' and f_d are as in ``shade``."""
    mu = p["mean"]
    wi, wo = _directions(mu, light_pos, eye, light_dir)
    Rsh = quat_to_rotmat(p["shade_rot"])
    wi_l = (Rsh @ wi[..., None])[..., 0]
    wo_l = (Rsh @ wo[..., None])[..., 0]
    fd = diffuse(wi_l[:, 2])
    hs = wi_l + wo_l
    hn = torch.linalg.norm(hs, dim=-1, keepdim=True)
    ok = hn > 1e-12
    ez = torch.tensor([0.0, 0.0, 1.0], dtype=DT).expand_as(hs)
    h = torch.where(ok, hs / torch.where(ok, hn, torch.ones_like(hn)), ez)
    Rb = quat_to_rotmat(p["basis_rot"])                # [K,3,3], rows x, y, z
    sig = torch.exp(p["basis_log_sigma"])             # [K,3]
    K = Rb.shape[0]
    hk = h[:, None, :].expand(-1, K, -1)
    G = angular_gaussian(hk, Rb[None, :, 0, :], Rb[None, :, 1, :], Rb[None, :, 2, :],
                         sig[None, :, 0], sig[None, :, 1], sig[None, :, 2])   # [N,K]
    fs = (p["basis_weight"] * G).sum(1)                # Eq. 6
    c = p["albedo"] * fd[:, None] + p["spec_albedo"] * fs[:, None]
    return {"c": c, "wi": wi, "wo": wo, "fd": fd, "h": h, "G": G}


def positional_encoding(x: torch.Tensor, bands: int = PE_BANDS) -> torch.Tensor:
    """Positional encoding of Sec. 4.2 / 4.3 with `bands` frequency bands:
    [x, sin(pi x), cos(pi x), sin(2 pi x), cos(2 pi x), ...,
    sin(2^(bands-1) pi x), cos(2^(bands-1) pi x)], each entry a block of the
    components of x (3 + 6 bands values for a 3-vector)."""
    out = [x]
    for k in range(bands):
        out.append(torch.sin((2.0 ** k) * math.pi * x))
        out.append(torch.cos((2.0 ** k) * math.pi * x))
    return torch.cat(out, -1)


def basis_mlp_inputs(p: Dict[str, torch.Tensor], T: torch.Tensor, wi: torch.Tensor, wo: torch.Tensor):
    """Inputs of the paper's MLPs: Phi(T, w_i; mu, l) (Sec. 4.2, Eq. 8) gets
    [T, PE(w_i), PE(mu), l] (61 values) and Psi(w_o; mu, l) (Sec. 4.3) gets
    [PE(w_o), PE(mu), l] (60 values); w_i, w_o and mu in world space, l the
    per-Gaussian 6-D latent shared by both."""
    pm = positional_encoding(p["mean"])
    phi_in = torch.cat([T[:, None], positional_encoding(wi), pm, p["latent"]], 1)
    psi_in = torch.cat([positional_encoding(wo), pm, p["latent"]], 1)
    return phi_in, psi_in


def mlp_forward(layers, x: torch.Tensor, slope: float = 0.0) -> torch.Tensor:
    """Dense layers, ReLU (slope = 0) or leaky ReLU with the given negative
    slope after each hidden layer, sigmoid at the output (Sec. 4.2 and 4.3).
    ``layers`` = [(W [out,in], b [out]), ...]."""
    hcur = x
    for i, (w, b) in enumerate(layers):
        hcur = hcur @ as_t(w).T + as_t(b)
        if i + 1 < len(layers):
            hcur = torch.where(hcur > 0, hcur, slope * hcur) if slope else torch.relu(hcur)
    return sigmoid(hcur)


# ------------------------------------------------------------ camera pass

def camera_pass(proj_c, cam_view, opacity, colour, tprime, resid, consts: Consts,
                tprime_err=None, band_rows: int = 8, pixels=None, flips=None, stop_flips=None,
                amb_keys: Optional[list] = None, stop_keys: Optional[list] = None):
    """Third splatting (Sec. 3 Eq. 2-3; Sec. 4, Fig. 2) toward the camera.

    Per pixel, hits sorted by view depth; T starts at 1; a hit that would
    take T below t_min stops the pixel before it contributes; otherwise
    S += c alpha T, Sh += T' alpha T, R += r alpha T, T *= (1 - alpha).
    Final = S * Sh + R (background 0). Returns images [C, P] over the
    requested pixels, T_final, and the per-pixel ambiguity bound.

    ``flips`` inverts hit decisions and ``stop_flips`` the stop decisions
    taken at the given pair keys (a hit whose T (1 - alpha) sits within the
    float32 error of t_min): both for decisions a float32 evaluation may
    take either way. The keys the error model flags (hit decisions of pairs
    reached before the pixel stops, and stop decisions) are appended to
    ``amb_keys`` and ``stop_keys`` when they are lists."""
    W, H = cam_view.width, cam_view.height
    if pixels is not None:
        chunks = [("pix", torch.as_tensor(pixels, dtype=torch.int64))]
    else:
        chunks = [("rows", (y, min(H, y + band_rows))) for y in range(0, H, band_rows)]
    outS, outSh, outR, outT, outAmb = [], [], [], [], []
    for kind, arg in chunks:
        e = pixel_entries(proj_c, W, H, opacity, consts,
                          rows=arg if kind == "rows" else None,
                          pixels=arg if kind == "pix" else None, flips=flips)
        P = e["n_pix"]
        if e["L"] == 0:
            outS.append(torch.zeros(3, P, dtype=DT)); outSh.append(torch.zeros(P, dtype=DT))
            outR.append(torch.zeros(3, P, dtype=DT)); outT.append(torch.ones(P, dtype=DT))
            outAmb.append(torch.zeros(P, dtype=DT))
            continue
        alpha, hit, gidp = e["alpha_pad"], e["hit_pad"], e["gid_pad"]
        prefix = _excl_prefix_product(1.0 - alpha)
        T_excl, T_incl = prefix[:, :-1], prefix[:, 1:]
        # the pixel stops before the first hit that would take T below
        # t_min; nothing after it is blended
        with torch.no_grad():
            stop = hit & (T_incl.detach() < consts.t_min)
            if stop_flips is not None and len(stop_flips):
                stop = stop ^ (hit & torch.isin(e["key_pad"], torch.as_tensor(stop_flips, dtype=torch.int64)))
            stopped = torch.cumsum(stop.to(torch.int64), 1) > 0
        inc = hit & ~stopped
        w = torch.where(inc, alpha * T_excl, torch.zeros_like(alpha))
        g = gidp.clamp_min(0)
        cpix = colour[g]                       # [P, L, 3]
        S = (w[..., None] * cpix).sum(1).T
        Sh = (w * tprime[g]).sum(1)
        R = (w[..., None] * resid[g]).sum(1).T
        Tfin = torch.where(inc, 1.0 - alpha, torch.ones_like(alpha)).prod(1)
        with torch.no_grad():
            amb, af = e["amb_pad"], e["alpha_full_pad"]
            Te = T_excl.detach()
            # relative float32 error of the transmittance in front of and
            # through each entry (products of the hits' factors)
            R_incl = torch.cumsum(e["t_relerr_pad"], 1)
            R_excl = R_incl - e["t_relerr_pad"]
            live = Te >= consts.t_min * (1 - R_excl)
            w_thr = torch.where(amb & live, af * Te, torch.zeros_like(af)).sum(1)
            Ti = T_incl.detach()
            near_stop = hit & ((Ti - consts.t_min).abs() <= R_incl * Ti) & (consts.t_min > 0)
            # only decisions the pixel reaches matter: hits before its stop
            reached = ~(torch.cumsum(stop.to(torch.int64), 1) - stop.to(torch.int64) > 0)
            near_stop = near_stop & reached
            w_stop = torch.where(near_stop, af * Te, torch.zeros_like(af)).sum(1)
            if amb_keys is not None:
                amb_keys.append(e["key_pad"][amb & live & reached])
            if stop_keys is not None:
                stop_keys.append(e["key_pad"][near_stop])
            cabs = torch.where(hit, colour.detach().abs().amax(1)[g], torch.zeros_like(af))
            cmax = cabs.amax(1).clamp_min(1.0)
            rmax = torch.where(hit, resid.detach().abs().amax(1)[g], torch.zeros_like(af)).amax(1)
            C = 2.0 * (2.0 * cmax + rmax + 1.0)
            ambw = C * (w_thr + w_stop)
            if tprime_err is not None:
                ambw = ambw + cmax * (w.detach() * tprime_err[g]).sum(1)
        outS.append(S); outSh.append(Sh); outR.append(R); outT.append(Tfin); outAmb.append(ambw)
    return (torch.cat(outS, 1), torch.cat(outSh, 0), torch.cat(outR, 1),
            torch.cat(outT, 0), torch.cat(outAmb, 0))


# ---------------------------------------------------------------- pipeline

def render(scene, cam_view, light_view, consts: Consts = Consts(),
           params: Optional[Dict[str, torch.Tensor]] = None,
           phi=None, psi=None, band_rows: int = 8, cam_pixels=None,
           light_pixels=None, light_flips=None, cam_flips=None, cam_stop_flips=None):
    """The full relit render for one camera and one point light (Sec. 4).

    1. activate raw parameters (Eq. 1; sigmoid opacity);
    2. shadow splatting toward the light (Sec. 4.2) -> T per Gaussian;
    3. shading (Sec. 4.1) -> c; Phi refines T -> T' (Eq. 8); Psi -> r
       (Sec. 4.3); a disabled MLP passes T through / gives r = 0;
    4. camera splatting of c, T', r and final = S * Sh + R (Fig. 2).

    ``phi``/``psi`` are lists of (W, b) (arrays or tensors) or None.
    ``params`` (from ``scene_tensors``) may carry requires_grad tensors.
    ``light_flips``, ``cam_flips`` and ``cam_stop_flips`` invert threshold
    decisions that the float32 error model flags (see ``shadow_pass`` and
    ``camera_pass``); the flagged pair keys are returned as
    "amb_light_keys", "amb_cam_keys" and "amb_stop_keys"."""
    p = params if params is not None else scene_tensors(scene)
    cov = covariance(p["log_scale"], p["rot"])
    opacity = sigmoid(p["opacity_logit"])
    light_pos = as_t(light_view.eye)
    proj_l = project(p["mean"], cov, light_view, consts, "dist")
    lk, ck, sk = [], [], []
    num, den, infl = shadow_pass(proj_l, light_view, opacity, consts,
                                 band_rows=band_rows, pixels=light_pixels, flips=light_flips, amb_keys=lk)
    T = shadow_values(num, den)
    with torch.no_grad():
        amb_T = torch.where(den > 0, infl / torch.where(den > 0, den, torch.ones_like(den)),
                            torch.where(infl > 0, torch.ones_like(infl), torch.zeros_like(infl)))
    # the paper's shared-basis appearance and MLP inputs when the scene has
    # them, else the isotropic per-Gaussian lobes and [T, feat] / [feat, w_i, w_o]
    basis = "basis_weight" in p
    shade_fn = shade_basis if basis else shade
    slope = LEAKY_SLOPE if basis else 0.0
    if is_ortho(light_view):
        sh = shade_fn(p, None, cam_view.eye, light_dir=np.asarray(light_view.eye) - np.asarray(light_view.target))
    else:
        sh = shade_fn(p, light_pos, cam_view.eye)

    def phi_input(t, q, wi):
        if basis:
            return basis_mlp_inputs(q, t, wi, sh["wo"])[0]
        return torch.cat([t[:, None], q["feat"]], 1)
    if phi is not None:
        tp = mlp_forward(phi, phi_input(T, p, sh["wi"]), slope)[:, 0]
        with torch.enable_grad():
            tq = T.detach().clone().requires_grad_(True)
            yq = mlp_forward(phi, phi_input(tq, {k: v.detach() for k, v in p.items()}, sh["wi"].detach()),
                             slope)[:, 0]
            dphi = torch.autograd.grad(yq.sum(), tq)[0].abs()
        amb_Tp = 2.0 * dphi * amb_T
    else:
        tp = T
        amb_Tp = amb_T
    if psi is not None:
        x_psi = basis_mlp_inputs(p, T, sh["wi"], sh["wo"])[1] if basis else torch.cat([p["feat"], sh["wi"], sh["wo"]], 1)
        r = mlp_forward(psi, x_psi, slope)
    else:
        r = torch.zeros_like(sh["c"])
    proj_c = project(p["mean"], cov, cam_view, consts, "z")
    S, Sh, R, Tfin, amb_px = camera_pass(proj_c, cam_view, opacity, sh["c"], tp, r, consts,
                                         tprime_err=amb_Tp.clamp_max(1.0),
                                         band_rows=band_rows, pixels=cam_pixels, flips=cam_flips,
                                         stop_flips=cam_stop_flips, amb_keys=ck, stop_keys=sk)
    final = S * Sh[None, :] + R
    cat = lambda x: torch.cat(x) if x else torch.zeros(0, dtype=torch.int64)  # noqa: E731
    return {"final": final, "S": S, "Sh": Sh, "R": R, "T_final": Tfin,
            "T": T, "num": num, "den": den, "Tp": tp, "c": sh["c"], "r": r,
            "amb_T": amb_T, "amb_px": amb_px, "proj_l": proj_l, "proj_c": proj_c,
            "opacity": opacity, "amb_light_keys": cat(lk), "amb_cam_keys": cat(ck),
            "amb_stop_keys": cat(sk)}


def render_env(scene, cam_view, light_views, weights, consts: Consts = Consts(), **kw) -> torch.Tensor:
    """Environment lighting (Sec. 4.5): the linear combination
    sum_k w_k final_k of the renders under directional lights (orthographic
    light views) sampled from the environment. Returns final [3, P]."""
    out = None
    for lv, w in zip(light_views, weights):
        f = render(scene, cam_view, lv, consts, **kw)["final"] * float(w)
        out = f if out is None else out + f
    return out


# --------------------------------------------------------------- training

def adam_step(param, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-15):
    """One Adam update (Kingma and Ba 2015; the optimiser of Sec. 4.4, with
    momentum beta1 = 0.9), float64: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2)
    g^2, p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t = step
    (1 for the first update). Returns (param, m, v)."""
    p, g = np.asarray(param, np.float64), np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def l1_loss(pred, target, scale: float):
    """The L1 term of the training loss (Sec. 4.4, Eq. 9): scale * sum
    |pred - target| over all elements, in float64, and its subgradient
    scale * sign(pred - target), taken as 0 where the two are equal.
    Returns (value, gradient array)."""
    d = np.asarray(pred, np.float64) - np.asarray(target, np.float64)
    return float(scale * np.abs(d).sum()), scale * np.sign(d)


# SSIM constants (Wang et al. 2004, the SSIM the loss of Sec. 4.4 refers
# to): an 11 x 11 Gaussian window of standard deviation 1.5, C1 = (0.01 L)^2,
# C2 = (0.03 L)^2 with dynamic range L = 1.
SSIM_WINDOW = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2
LOSS_LAMBDA = 0.2        # Sec. 4.4: weight of the D-SSIM term


def ssim_window() -> torch.Tensor:
    """The normalised 11 x 11 Gaussian window (outer product of a normalised
    1-D Gaussian with sigma 1.5), float64."""
    r = SSIM_WINDOW // 2
    x = torch.arange(-r, r + 1, dtype=DT)
    g = torch.exp(-x * x / (2 * SSIM_SIGMA ** 2))
    g = g / g.sum()
    return g[:, None] * g[None, :]


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Per-pixel SSIM of images x, y [C, H, W] (float64): local means,
    variances and covariance from the Gaussian window centred on the pixel,
    zero outside the image, each channel on its own:
    s = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2))."""
    w = ssim_window()
    C = x.shape[0]
    k = w[None, None].expand(C, 1, *w.shape)
    pad = SSIM_WINDOW // 2
    blur = lambda t: torch.nn.functional.conv2d(t[None], k, padding=pad, groups=C)[0]  # noqa: E731
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def dssim_loss(pred, target, scale: float):
    """The D-SSIM term of the training loss (Sec. 4.4, Eq. 9; the D-SSIM of
    the Gaussian-splatting loss the paper adopts): scale * sum over channels
    and pixels of (1 - SSIM). Returns (value, gradient array) in float64;
    scale = lambda / (C H W) gives lambda times the mean D-SSIM."""
    x = as_t(pred).clone().requires_grad_(True)
    val = scale * (1.0 - ssim_map(x, as_t(target))).sum()
    val.backward()
    return float(val.detach()), x.grad.numpy()


def render_images(out: Dict, view) -> Dict[str, np.ndarray]:
    """Reshape full-frame outputs of ``render`` to [C, H, W] numpy arrays."""
    H, W = view.height, view.width
    return {
        "final": out["final"].detach().reshape(3, H, W).numpy(),
        "S": out["S"].detach().reshape(3, H, W).numpy(),
        "Sh": out["Sh"].detach().reshape(H, W).numpy(),
        "R": out["R"].detach().reshape(3, H, W).numpy(),
        "T_final": out["T_final"].detach().reshape(H, W).numpy(),
        "amb_px": out["amb_px"].detach().reshape(H, W).numpy(),
    }
