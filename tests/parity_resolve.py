"""Decision resolution for GPU parity tests (helper, not a test module).

A few threshold decisions of a render hang on float32 rounding: pairs whose
power lies within the oracle's error margin of the cut-off (or the alpha
minimum), and stop decisions whose transmittance lies within the float32
error of t_min. The oracle flags them (``amb_light_keys``, ``amb_cam_keys``,
``amb_stop_keys``); either outcome is a correct evaluation of the method.

Instead of leaving the outputs that depend on them out of the comparison,
``resolve`` finds the outcome the GPU took for each flagged decision and
renders the oracle with exactly those decisions, so that every output can
then be compared:

- light decisions change the shadow values of the Gaussians on that light
  ray. Per ray, each subset of its flagged pairs is evaluated with the
  oracle's own shadow pass restricted to the ray's pixel, and the subset
  whose shadow values are closest to the GPU's is taken (rays are visited
  twice, so rays sharing Gaussians settle jointly);
- camera decisions change only their own pixel; per pixel each subset of its
  flagged decisions is evaluated with the oracle's camera pass restricted to
  that pixel and the closest to the GPU's pixel is taken.

Only flagged decisions can be chosen, so a GPU that takes an unflagged
decision the other way, or computes anything else differently, still fails
the comparison.
"""
from __future__ import annotations

import itertools
from typing import Dict, Optional

import numpy as np
import torch

import oracle as O

MAX_GROUP = 4        # at most 2^4 outcome combinations per ray or pixel


def _subsets(keys):
    keys = list(keys)
    for r in range(len(keys) + 1):
        for c in itertools.combinations(keys, r):
            yield list(c)


def _group(keys: torch.Tensor, npx: int):
    out: Dict[int, list] = {}
    for k in torch.unique(keys).tolist():
        out.setdefault(k % npx, []).append(k)
    return out


def restrict(pr, op, pixels, W: int, consts):
    """The Gaussians whose oracle candidate rectangle (the bounding box of
    power >= -cutoff, slightly widened, as ``O.pixel_entries`` forms it)
    meets the bounding box of the flat pixel indices `pixels` of a W-wide
    view: (ids, projection and opacity restricted to them). A pass over
    those pixels gives the same sums with these Gaussians as with all (no
    other one can reach them); ids are ascending, so ties in depth keep the
    same order."""
    pixels = torch.as_tensor(pixels)
    py, px = pixels // W, pixels % W
    x0, x1, y0, y1 = int(px.min()), int(px.max()), int(py.min()), int(py.max())
    cut = O.CANDIDATE_CUT(consts.cutoff)
    u, v = pr["u"].detach(), pr["v"].detach()
    if np.isinf(cut):
        touch = pr["valid"]
    else:
        hx = torch.sqrt(2 * cut * pr["cov2"][:, 0].detach().clamp_min(0)) + 1.0
        hy = torch.sqrt(2 * cut * pr["cov2"][:, 2].detach().clamp_min(0)) + 1.0
        touch = pr["valid"] & (u + hx >= x0) & (u - hx <= x1 + 1) & (v + hy >= y0) & (v - hy <= y1 + 1)
    ids = torch.nonzero(touch).flatten()
    return ids, {k: t[ids] for k, t in pr.items()}, op[ids]


def shadow_pass_near(pr, light, op, consts, pixels, flips=None, pairs: bool = False):
    """``O.shadow_pass`` over `pixels` run on only the Gaussians that can
    reach them (``restrict``); same results, returned in the caller's
    numbering: (num, den, infl) over all Gaussians and the flagged pair
    keys (Gaussian index * W * H + pixel); with ``pairs`` also every hit's
    (Gaussian, pixel, num term, den term)."""
    W, H = light.width, light.height
    n = op.shape[0]
    ids, sub, sop = restrict(pr, op, pixels, W, consts)
    npx = W * H
    local_flips = None
    if flips is not None and len(flips):
        f = torch.as_tensor(flips, dtype=torch.int64)
        pos = torch.full((n,), -1, dtype=torch.int64)
        pos[ids] = torch.arange(len(ids))
        g = pos[f // npx]
        local_flips = (g[g >= 0] * npx + (f % npx)[g >= 0]).tolist()
    keys, po = [], ([] if pairs else None)
    a, b, c = O.shadow_pass(sub, light, sop, consts, pixels=torch.as_tensor(pixels), flips=local_flips,
                            amb_keys=keys, pair_out=po)
    num = torch.zeros(n, dtype=torch.float64).index_add(0, ids, a.detach())
    den = torch.zeros(n, dtype=torch.float64).index_add(0, ids, b.detach())
    infl = torch.zeros(n, dtype=torch.float64).index_add(0, ids, c)
    keys = torch.cat(keys) if keys else torch.zeros(0, dtype=torch.int64)
    keys = ids[keys // npx] * npx + keys % npx
    if not pairs:
        return num, den, infl, keys
    if po:
        g, px, tn, td = (torch.cat([t[i] for t in po]) for i in range(4))
        g = ids[g]
    else:
        g = px = torch.zeros(0, dtype=torch.int64)
        tn = td = torch.zeros(0, dtype=torch.float64)
    return num, den, infl, keys, (g, px, tn, td)


def _per_pixel(terms, want_pixels):
    """{pixel: (Gaussians, num terms, den terms)} from a pass's pair terms."""
    g, px, tn, td = terms
    out = {}
    if g.numel() == 0:
        return out
    o = torch.argsort(px, stable=True)
    g, px, tn, td = g[o], px[o], tn[o], td[o]
    uniq, counts = torch.unique_consecutive(px, return_counts=True)
    start = 0
    for p, c in zip(uniq.tolist(), counts.tolist()):
        if p in want_pixels:
            out[p] = (g[start:start + c].numpy(), tn[start:start + c].numpy(), td[start:start + c].numpy())
        start += c
    return out


def _delta(base, alt):
    """Sparse per-Gaussian change from the terms `base` to `alt` of one ray:
    (Gaussians, d num, d den)."""
    gb, nb, db = base
    ga, na, da = alt
    idx = np.union1d(gb, ga)
    dn = np.zeros(len(idx))
    dd = np.zeros(len(idx))
    np.add.at(dn, np.searchsorted(idx, ga), na)
    np.add.at(dd, np.searchsorted(idx, ga), da)
    np.add.at(dn, np.searchsorted(idx, gb), -nb)
    np.add.at(dd, np.searchsorted(idx, gb), -db)
    return idx, dn, dd


def resolve_light(prl, light, op, consts, T_gpu: np.ndarray, num0, den0, amb_keys: torch.Tensor,
                  observed: Optional[np.ndarray] = None, max_per_ray: int = 64):
    """The GPU's outcome of each flagged light decision. num0/den0: the
    oracle's sums without flips; T_gpu: the GPU's shadow values; observed:
    the Gaussians whose GPU shadow value the oracle's sums describe (all by
    default; fewer when the sums cover only part of the light image).

    Each flagged pair is a decision of its own. The change of flipping it is
    measured by the oracle (one pass per j flipping the j-th flagged pair of
    every ray), the decisions are chosen by coordinate descent on the
    largest shadow-value error of the Gaussians they touch (changes of two
    flips on one ray taken as additive for the choice), and the comparison
    afterwards renders the chosen decisions exactly. Returns (flips,
    unresolved Gaussians mask, number flagged)."""
    n = len(T_gpu)
    W, H = light.width, light.height
    groups = _group(amb_keys, W * H)
    obs = np.ones(n, bool) if observed is None else observed
    unresolved = np.zeros(n, bool)
    flips: list = []
    if not groups:
        return flips, unresolved, 0
    num0 = np.asarray(num0, np.float64)
    den0 = np.asarray(den0, np.float64)
    pixels = sorted(groups)
    pset = set(pixels)
    empty = (np.zeros(0, np.int64), np.zeros(0), np.zeros(0))
    with torch.no_grad():
        base = _per_pixel(shadow_pass_near(prl, light, op, consts, pixels, pairs=True)[4], pset)
        single = []
        for j in range(max_per_ray):
            pj = [p for p in pixels if max_per_ray >= len(groups[p]) > j]
            if not pj:
                break
            fj = [groups[p][j] for p in pj]
            single.append(_per_pixel(shadow_pass_near(prl, light, op, consts, pj, flips=fj, pairs=True)[4],
                                     set(pj)))
    units = []       # (key, touched Gaussians, d num, d den)
    for pix in pixels:
        keys = groups[pix]
        b = base.get(pix, empty)
        if len(keys) > max_per_ray:
            unresolved[b[0]] |= obs[b[0]]        # every Gaussian on the ray
            continue
        for j, key in enumerate(keys):
            idx, dn, dd = _delta(b, single[j].get(pix, empty))
            keep = obs[idx]
            if keep.any():
                units.append((key, idx[keep], dn[keep], dd[keep]))
    on = [False] * len(units)
    tot_n = np.zeros(n)
    tot_d = np.zeros(n)
    for _ in range(3):
        changed = False
        for u, (key, idx, dn, dd) in enumerate(units):
            num = num0[idx] + tot_n[idx] - (dn if on[u] else 0.0)    # with every other decision as chosen
            den = den0[idx] + tot_d[idx] - (dd if on[u] else 0.0)
            errs = []
            for nn, d2 in ((num, den), (num + dn, den + dd)):
                Tc = np.where(d2 > 0, nn / np.where(d2 > 0, d2, 1.0), 1.0)
                errs.append(np.abs(Tc - T_gpu[idx]).max())
            want = errs[1] < errs[0]
            if want != on[u]:
                sgn = 1.0 if want else -1.0
                tot_n[idx] += sgn * dn
                tot_d[idx] += sgn * dd
                on[u] = want
                changed = True
        if not changed:
            break
    flips = [units[u][0] for u in range(len(units)) if on[u]]
    return flips, unresolved, int(sum(len(g) for g in groups.values()))


def resolve_camera(prc, cam, op, c, tp, r, consts, hit_keys, stop_keys, gpu_px: Dict[str, np.ndarray],
                   order):
    """The GPU's outcome of each flagged camera decision (pair hits and stop
    decisions), pixel by pixel. gpu_px: GPU outputs over the pixels `order`
    (flat indices). Returns (hit flips, stop flips, unresolved pixel mask
    over `order`)."""
    W, H = cam.width, cam.height
    px_items: Dict[int, list] = {}
    for k in torch.unique(torch.as_tensor(hit_keys, dtype=torch.int64)).tolist():
        px_items.setdefault(k % (W * H), []).append(("hit", k))
    for k in torch.unique(torch.as_tensor(stop_keys, dtype=torch.int64)).tolist():
        px_items.setdefault(k % (W * H), []).append(("stop", k))
    where = {p: i for i, p in enumerate(list(order))}
    unresolved = np.zeros(len(where), bool)
    cam_flips, stop_flips = [], []
    for pix, items in px_items.items():
        i = where[pix]
        if len(items) > MAX_GROUP:
            unresolved[i] = True
            continue
        g = np.concatenate([gpu_px["final"][:, i], gpu_px["S"][:, i], [gpu_px["Sh"][i]],
                            gpu_px["R"][:, i], [gpu_px["T_final"][i]]])
        best, best_err = [], np.inf
        for sub in _subsets(items):
            hf = [k for kind, k in sub if kind == "hit"]
            sf = [k for kind, k in sub if kind == "stop"]
            with torch.no_grad():
                S, Sh, R, Tf, _ = O.camera_pass(prc, cam, op, c, tp, r, consts, pixels=torch.tensor([pix]),
                                                flips=hf, stop_flips=sf)
            fin = (S * Sh[None, :] + R)[:, 0]
            v = np.concatenate([fin.numpy(), S[:, 0].numpy(), Sh.numpy(), R[:, 0].numpy(), Tf.numpy()])
            err = np.abs(v - g).max()
            if err < best_err - 1e-12:
                best, best_err = sub, err
        cam_flips += [k for kind, k in best if kind == "hit"]
        stop_flips += [k for kind, k in best if kind == "stop"]
    return cam_flips, stop_flips, unresolved


def resolve(sc, cam, light, consts, phi, psi, T_gpu: np.ndarray, gpu_px: Dict[str, np.ndarray],
            cam_pixels: Optional[torch.Tensor] = None, light_pixels: Optional[torch.Tensor] = None,
            params=None):
    """Oracle render whose flagged decisions follow the GPU's.

    T_gpu: the GPU's shadow values [n]. gpu_px: the GPU's camera outputs over
    the compared pixels, "final" [3, P], "S" [3, P], "Sh" [P], "R" [3, P],
    "T_final" [P] in the order of ``cam_pixels`` (default: every pixel in
    row-major order). Returns (ref, info) with ref the oracle's render (as
    ``O.render``) and info the counts of flagged and flipped decisions and
    of the rays / pixels whose flagged decisions were too many to resolve
    (``unresolved_T`` / ``unresolved_px`` masks over Gaussians / compared
    pixels)."""
    kw = dict(phi=phi, psi=psi, cam_pixels=cam_pixels, light_pixels=light_pixels, params=params)
    with torch.no_grad():
        ref0 = O.render(sc, cam, light, consts, **kw)
    info = {}
    light_flips, unresolved_T, info["light_flagged"] = resolve_light(
        ref0["proj_l"], light, ref0["opacity"].detach(), consts, T_gpu, ref0["num"].detach().numpy(),
        ref0["den"].detach().numpy(), ref0["amb_light_keys"])
    info["light_flipped"] = len(light_flips)
    with torch.no_grad():
        ref1 = O.render(sc, cam, light, consts, light_flips=light_flips, **kw)
    hit_keys, stop_keys = ref1["amb_cam_keys"], ref1["amb_stop_keys"]
    info["cam_flagged"] = int(torch.unique(hit_keys).numel())
    info["stop_flagged"] = int(torch.unique(stop_keys).numel())
    order = (torch.arange(cam.width * cam.height) if cam_pixels is None else torch.as_tensor(cam_pixels)).tolist()
    cam_flips, stop_flips, unresolved_px = resolve_camera(
        ref1["proj_c"], cam, ref1["opacity"].detach(), ref1["c"].detach(), ref1["Tp"].detach(),
        ref1["r"].detach(), consts, hit_keys, stop_keys, gpu_px, order)
    info["cam_flipped"], info["stop_flipped"] = len(cam_flips), len(stop_flips)
    ref = O.render(sc, cam, light, consts, light_flips=light_flips, cam_flips=cam_flips,
                   cam_stop_flips=stop_flips, **kw)
    info["unresolved_T"] = unresolved_T
    info["unresolved_px"] = unresolved_px
    info["flips"] = (light_flips, cam_flips, stop_flips)
    return ref, info


def describe(info) -> str:
    return (f"light decisions flagged {info['light_flagged']} flipped {info['light_flipped']}, camera "
            f"{info['cam_flagged']}/{info['cam_flipped']}, stop {info['stop_flagged']}/{info['stop_flipped']}, "
            f"unresolved Gaussians {int(info['unresolved_T'].sum())}, pixels {int(info['unresolved_px'].sum())}")
