"""Parity on the dense "fluffy" scene at full size: 1,500,000 Gaussians
(70 % low-opacity needles filling the cube, 30 % on the shell), camera
1024x1024 at 40 deg, light splat 2048x2048 at 60 deg, default Renderer.

Tile lists here run to tens of thousands of entries and few rays go dark,
so every stage runs its long-list paths. The oracle checks what it can
compute piece by piece:
  - the pair count of every tile of both views, bit for bit, from the
    oracle's tile rectangles of the GPU's integer extents;
  - the full sorted lists (ids and keys) of sampled tiles, bit for bit,
    against the oracle's brute-force binning of the splats covering them;
  - every Gaussian's colour c, refined shadow T' and residual r, given the
    GPU's shadow values T;
  - the shadow value T of the Gaussians whose whole light footprint lies
    inside a 48x48 light crop (the oracle's shadow pass is additive over
    pixels, so it runs in 16x16 blocks);
  - the shadow denominator of sampled large elongated splats (the banded
    path) and other splats, each from a one-Gaussian oracle pass, and the
    shadow values of the thinnest banded needles;
  - two 16x16 patches of the camera images, given the GPU's T.
Tolerance 1e-4 max abs over every checked output; the threshold decisions
the oracle flags as float32-ambiguous follow the GPU's
(tests/parity_resolve.py)."""
import time

import numpy as np
import pytest
import torch

import oracle as O
from oracle.gs3_oracle import AMB_BUDGET
from paper_2410_11419_amd import synth
from parity_resolve import resolve_camera, resolve_light, restrict, shadow_pass_near

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def run():
    assert torch.cuda.is_available()
    from paper_2410_11419_amd import gs3
    t0 = time.perf_counter()
    sc = synth.scene_fluffy()
    cam, light = synth.fluffy_pairs(1)[0]
    ds = gs3.DeviceScene.from_host(sc)
    rnd = gs3.Renderer(ds)
    out = rnd.render(cam, light)
    torch.cuda.synchronize()
    print(f"\nfluffy scene built and rendered in {time.perf_counter() - t0:.1f} s", flush=True)
    res = {k: v.detach().cpu().numpy() for k, v in out.items()}
    views = {}
    for role, vb in (("light", rnd.vbs[("light", 2048, 2048)]), ("cam", rnd.vbs[("cam", 1024, 1024)])):
        ts, te, ids, keys = gs3.gs3_view_lists(vb)
        _, _, _, depth, ext = gs3.gs3_view_splats(vb)
        views[role] = dict(ts=ts.cpu().numpy().astype(np.int64), te=te.cpu().numpy().astype(np.int64),
                           ids=ids, keys=keys, ext=ext.cpu().numpy().astype(np.int64),
                           depth=depth.cpu().numpy())
    p = O.scene_tensors(sc)
    cov = O.covariance(p["log_scale"], p["rot"])
    op = O.sigmoid(p["opacity_logit"])
    k = O.Consts()
    prl = O.project(p["mean"], cov, light, k, "dist")
    prc = O.project(p["mean"], cov, cam, k, "z")
    return dict(sc=sc, cam=cam, light=light, res=res, views=views, p=p, op=op, prl=prl, prc=prc, k=k)


def _rect_counts(ext, W, H):
    """Per-tile number of oracle tile rectangles covering it (2-D difference
    array over the rectangles of ``O.tile_rects``)."""
    x0, x1, y0, y1, empty = O.tile_rects(ext[0], ext[1], ext[2], ext[3], W, H)
    tx, ty = (W + 15) // 16, (H + 15) // 16
    keep = ~empty
    x0, x1, y0, y1 = x0[keep], x1[keep], y0[keep], y1[keep]
    diff = np.zeros((ty + 1, tx + 1), np.int64)
    np.add.at(diff, (y0, x0), 1)
    np.add.at(diff, (y0, x1 + 1), -1)
    np.add.at(diff, (y1 + 1, x0), -1)
    np.add.at(diff, (y1 + 1, x1 + 1), 1)
    return diff.cumsum(0).cumsum(1)[:ty, :tx].ravel()


def _oracle_tile_list(ext, depth, W, H, tile):
    """The oracle's list of one tile: brute-force binning of the splats whose
    rectangle covers that tile (no other splat can appear in its list)."""
    x0, x1, y0, y1, empty = O.tile_rects(ext[0], ext[1], ext[2], ext[3], W, H)
    tx = (W + 15) // 16
    gx, gy = tile % tx, tile // tx
    sub = np.nonzero(~empty & (x0 <= gx) & (gx <= x1) & (y0 <= gy) & (gy <= y1))[0]
    counts, ids, keys = O.bin_tiles(ext[0][sub], ext[1][sub], ext[2][sub], ext[3][sub], depth[sub], W, H)
    first = int(counts[:tile].sum())
    return sub[ids[first:first + counts[tile]]], keys[first:first + counts[tile]]


@pytest.mark.parametrize("role", ["light", "cam"])
def test_fluffy_lists_bit_exact(run, role):
    V = run["views"][role]
    view = run["light"] if role == "light" else run["cam"]
    W, H = view.width, view.height
    counts = V["te"] - V["ts"]
    np.testing.assert_array_equal(counts, _rect_counts(V["ext"], W, H))
    rng = np.random.default_rng(0)
    nonempty = np.nonzero(counts)[0]
    tiles = {int(np.argmax(counts)), int(nonempty[np.argsort(counts[nonempty])[nonempty.size // 2]]),
             int(counts.size - 1)}
    tiles |= {int(t) for t in rng.choice(nonempty, 3, replace=False)}
    for t in sorted(tiles):
        o_ids, o_keys = _oracle_tile_list(V["ext"], V["depth"], W, H, t)
        s, e = int(V["ts"][t]), int(V["te"][t])
        np.testing.assert_array_equal(V["ids"][s:e].cpu().numpy(), o_ids)
        np.testing.assert_array_equal(V["keys"][s:e].cpu().numpy().view(np.uint64), o_keys)
    print(f"[{role}] {int(counts.sum())} pairs over {counts.size} tiles, longest list {int(counts.max())}; "
          f"lists of tiles {sorted(tiles)} checked")


def test_fluffy_appearance_given_T(run):
    sc, p, res = run["sc"], run["p"], run["res"]
    n = sc.n
    T = torch.as_tensor(res["T"][:n].astype(np.float64))
    sh = O.shade(p, run["light"].eye, run["cam"].eye)
    tp = O.mlp_forward(sc.phi.layers, torch.cat([T[:, None], p["feat"]], 1))[:, 0]
    r = O.mlp_forward(sc.psi.layers, torch.cat([p["feat"], sh["wi"], sh["wo"]], 1))
    col = res["colour"][:, :n]
    err_c = np.abs(col[0:3] - sh["c"].numpy().T).max()
    err_tp = np.abs(col[3] - tp.numpy()).max()
    err_r = np.abs(col[4:7] - r.numpy().T).max()
    print(f"colour {err_c:.2e}, T' {err_tp:.2e}, r {err_r:.2e} over {n} Gaussians")
    assert err_c <= TOL and err_tp <= TOL and err_r <= TOL


def test_fluffy_shadow_crop(run):
    """Shadow values of the Gaussians wholly inside a 48x48 light crop; the
    crop rays' flagged decisions follow the GPU's (tests/parity_resolve.py).
    The oracle runs on the Gaussians that can reach the crop (no other one
    changes a crop pixel)."""
    light, prl, op, k = run["light"], run["prl"], run["op"], run["k"]
    n = run["sc"].n
    ix, iy, rx, ry = [np.asarray(a) for a in O.splat_extent(prl, op, k)]
    x0, y0, w = 1000, 1000, 48
    ys, xs = np.meshgrid(np.arange(y0, y0 + w), np.arange(x0, x0 + w), indexing="ij")
    crop = torch.as_tensor((ys * light.width + xs).ravel())
    ids, sub, sop = restrict(prl, op, crop, light.width, k)
    idn = ids.numpy()
    m = len(idn)
    inside = ((rx >= 0) & (ix - rx >= x0) & (ix + rx < x0 + w) & (iy - ry >= y0) & (iy + ry < y0 + w))[idn]
    T_g = run["res"]["T"][:n][idn]
    print(f"\n  {m} of {n} Gaussians reach the crop", flush=True)
    num = torch.zeros(m, dtype=torch.float64)
    den = torch.zeros(m, dtype=torch.float64)
    infl = torch.zeros(m, dtype=torch.float64)
    keys = []
    t0 = time.perf_counter()
    for by in range(y0, y0 + w, 16):
        for bx in range(x0, x0 + w, 16):
            ys, xs = np.meshgrid(np.arange(by, by + 16), np.arange(bx, bx + 16), indexing="ij")
            pix = torch.as_tensor((ys * light.width + xs).ravel())
            a, b, c, kk = shadow_pass_near(sub, light, sop, k, pix)
            keys.append(kk)
            num += a
            den += b
            infl += c
        print(f"  crop rows {by}..{by + 15} done ({time.perf_counter() - t0:.0f} s)", flush=True)
    keys = torch.cat(keys) if keys else torch.zeros(0, dtype=torch.int64)
    flips, unresolved, nflag = resolve_light(sub, light, sop, k, T_g, num.numpy(), den.numpy(), keys,
                                             observed=inside)
    assert not unresolved.any()
    if flips:
        # the flipped pairs' rays again, with the GPU's decisions
        fpix = torch.unique(torch.as_tensor(flips) % (light.width * light.height))
        a0, b0, _, _ = shadow_pass_near(sub, light, sop, k, fpix)
        a1, b1, _, _ = shadow_pass_near(sub, light, sop, k, fpix, flips=flips)
        num, den = num - a0 + a1, den - b0 + b1
    T_o = O.shadow_values(num, den).numpy()
    sel = inside & (den.numpy() > 0)
    bmask = sel & ((infl / torch.where(den > 0, den, torch.ones_like(den))).numpy() > AMB_BUDGET)
    err = np.abs(T_g[sel] - T_o[sel])
    worst = float(err.max()) if sel.any() else 0.0
    wb = float(np.abs(T_g[bmask] - T_o[bmask]).max()) if bmask.any() else 0.0
    print(f"shadow values of {int(sel.sum())} Gaussians inside a {w}x{w} light crop: max err {worst:.2e}; "
          f"flagged light decisions {nflag}, flipped {len(flips)}; bound-flagged {int(bmask.sum())} "
          f"(max err {wb:.2e}); oracle {time.perf_counter() - t0:.0f} s")
    assert sel.sum() >= 20
    assert worst <= TOL


def _subset_projection(pr, idx):
    return {key: v[idx] for key, v in pr.items()}


def test_fluffy_banded_denominator(run):
    """The shadow denominator den_j = sum of beta over the light pixels
    Gaussian j hits depends on j alone, so a one-Gaussian oracle pass gives
    it exactly. Checked for a sample of the large elongated splats whose
    denominator narrows each tile row to the ellipse's own band (16 tiles or
    more, bounding box over 2.5x the ellipse) and a sample of the others.
    Flagged pairs of j may add or drop their beta; that much slack is
    allowed per flagged pair, and counted. Then the shadow values T of the
    thinnest banded needles, from a full oracle pass over the light pixels
    each one reaches (its T depends on those rays only)."""
    light, prl, op, k, res = run["light"], run["prl"], run["op"], run["k"], run["res"]
    n = run["sc"].n
    ix, iy, rx, ry = O.splat_extent(prl, op, k)
    x0, x1, y0, y1, empty = O.tile_rects(ix, iy, rx, ry, light.width, light.height)
    tiles = (x1 - x0 + 1) * (y1 - y0 + 1)
    con = prl["conic"].numpy()
    det = con[:, 0] * con[:, 2] - con[:, 1] ** 2
    banded = (~empty) & (tiles >= 16) & (con[:, 0] * con[:, 2] > 4 * det)
    rng = np.random.default_rng(5)
    b_ids = rng.choice(np.nonzero(banded)[0], 300, replace=False)
    o_ids = rng.choice(np.nonzero(~banded & ~empty)[0], 100, replace=False)
    ids = np.concatenate([b_ids, o_ids])
    sub = _subset_projection(prl, torch.as_tensor(ids))
    keys = []
    t0 = time.perf_counter()
    den_err = torch.zeros(len(ids), dtype=torch.float64)
    _, den_o, _ = O.shadow_pass(sub, light, op[ids], k, amb_keys=keys, den_err=den_err)
    keys = torch.cat(keys) if keys else torch.zeros(0, dtype=torch.int64)
    den_o = den_o.numpy()
    den_err = den_err.numpy()
    den_g = res["num_den"][1, :n][ids].astype(np.float64)
    nflag = np.bincount((keys // (light.width * light.height)).numpy(), minlength=len(ids)) if keys.numel() else \
        np.zeros(len(ids), np.int64)
    pth = O.hit_threshold(op[ids], k).numpy()
    slack = nflag * np.exp(-pth) * 1.01
    err = np.abs(den_g - den_o)
    # flagged pairs may add or drop their beta; every beta carries the float32
    # error of its power (large for thin needles, whose quadratic terms
    # cancel); the float32 sum adds a few ulp
    tol = 2e-6 * den_o + slack + den_err + 1e-7
    print(f"den of {len(b_ids)} banded and {len(o_ids)} other Gaussians: max rel err "
          f"{float((err / np.maximum(den_o, 1e-30)).max()):.2e}, max err / tolerance {float((err / tol).max()):.2f}; "
          f"Gaussians with flagged pairs {int((nflag > 0).sum())}; largest float32 bound of a den "
          f"{float((den_err / np.maximum(den_o, 1e-30)).max()):.1e} relative; oracle {time.perf_counter() - t0:.0f} s")
    for i in np.nonzero(err > tol)[0]:
        print(f"  Gaussian {ids[i]} ({'banded' if i < len(b_ids) else 'other'}): den gpu {den_g[i]:.6f} oracle "
              f"{den_o[i]:.6f}, flagged pairs {nflag[i]}, slack {slack[i]:.2e}")
    assert (den_o[:len(b_ids)] > 0).all()
    assert (err <= tol).all(), np.nonzero(err > tol)
    # shadow values of the thinnest banded needles
    pth_all = O.hit_threshold(op, k).numpy()
    ell = np.pi * 2 * pth_all / np.sqrt(np.maximum(det, 1e-30))
    # the most lit thin needles (few rays in this dense volume stay lit), so
    # the check has occluders to get right and a value to get
    T_g = res["T"][:n]
    cand = np.nonzero(banded & (ell > 60) & (ell < 800) & (res["num_den"][1, :n] > 0) &
                      (T_g > 1e-3) & (T_g < 0.999))[0]
    needles = cand[np.argsort(-T_g[cand])[:4]]
    worst = 0.0
    for j in needles:
        # the light pixels the needle hits, or may hit by rounding
        xa, xb = max(int(ix[j] - rx[j]), 0), min(int(ix[j] + rx[j]), light.width - 1)
        ya, yb = max(int(iy[j] - ry[j]), 0), min(int(iy[j] + ry[j]), light.height - 1)
        ys, xs = np.meshgrid(np.arange(ya, yb + 1), np.arange(xa, xb + 1), indexing="ij")
        box = torch.as_tensor((ys * light.width + xs).ravel())
        e = O.pixel_entries(_subset_projection(prl, torch.as_tensor([j])), light.width, light.height, op[[j]], k,
                            pixels=box)
        pix = box[(e["hit_pad"][:, 0] | e["amb_pad"][:, 0])]
        ids, sub, sop = restrict(prl, op, pix, light.width, k)
        jj = int(torch.nonzero(ids == int(j))[0])
        keys = []
        num, den, _ = O.shadow_pass(sub, light, sop, k, pixels=pix, amb_keys=keys)
        keys = torch.cat(keys) if keys else torch.zeros(0, dtype=torch.int64)
        obs = np.zeros(len(ids), bool)
        obs[jj] = True
        flips, unresolved, _ = resolve_light(sub, light, sop, k, T_g[ids.numpy()], num.numpy(), den.numpy(), keys,
                                             observed=obs)
        if flips:
            num, den, _ = O.shadow_pass(sub, light, sop, k, pixels=pix, flips=flips)
        T_o = float(O.shadow_values(num, den)[jj])
        worst = max(worst, abs(T_o - float(T_g[j])))
        print(f"  needle {j}: {pix.numel()} light pixels, T gpu {float(T_g[j]):.6f} oracle {T_o:.6f}", flush=True)
    assert len(needles) == 4
    assert worst <= TOL


def test_fluffy_camera_patches(run):
    """Two 16x16 camera patches given the GPU's T, every pixel, with the
    flagged camera decisions following the GPU's."""
    sc, p, res, cam, prc, op, k = run["sc"], run["p"], run["res"], run["cam"], run["prc"], run["op"], run["k"]
    n = sc.n
    T = torch.as_tensor(res["T"][:n].astype(np.float64))
    sh = O.shade(p, run["light"].eye, cam.eye)
    tp = O.mlp_forward(sc.phi.layers, torch.cat([T[:, None], p["feat"]], 1))[:, 0]
    r = O.mlp_forward(sc.psi.layers, torch.cat([p["feat"], sh["wi"], sh["wo"]], 1))
    worst = {}
    n_bound = flagged = flipped = 0
    for (x0, y0) in ((504, 504), (300, 640)):
        w = 16
        ys, xs = np.meshgrid(np.arange(y0, y0 + w), np.arange(x0, x0 + w), indexing="ij")
        pix = torch.as_tensor((ys * cam.width + xs).ravel())
        gpu = {"S": res["S"][:, ys, xs].reshape(3, -1), "Sh": res["Sh"][ys, xs].reshape(-1),
               "R": res["R"][:, ys, xs].reshape(3, -1), "final": res["final"][:, ys, xs].reshape(3, -1),
               "T_final": res["T_final"][ys, xs].reshape(-1)}
        ids, sub, sop = restrict(prc, op, pix, cam.width, k)
        sc_c, sc_tp, sc_r = sh["c"][ids], tp[ids], r[ids]
        hk, sk = [], []
        S, Sh, R, Tf, amb = O.camera_pass(sub, cam, sop, sc_c, sc_tp, sc_r, k, pixels=pix, amb_keys=hk, stop_keys=sk)
        hk = torch.cat(hk) if hk else torch.zeros(0, dtype=torch.int64)
        sk = torch.cat(sk) if sk else torch.zeros(0, dtype=torch.int64)
        cf, sf, unresolved = resolve_camera(sub, cam, sop, sc_c, sc_tp, sc_r, k, hk, sk, gpu, pix.tolist())
        assert not unresolved.any()
        flagged += int(torch.unique(hk).numel() + torch.unique(sk).numel())
        flipped += len(cf) + len(sf)
        if cf or sf:
            S, Sh, R, Tf, _ = O.camera_pass(sub, cam, sop, sc_c, sc_tp, sc_r, k, pixels=pix, flips=cf, stop_flips=sf)
        print(f"  patch ({x0}, {y0}): {len(ids)} Gaussians reach it", flush=True)
        n_bound += int((amb.numpy() > AMB_BUDGET).sum())
        final = (S * Sh[None, :] + R).numpy()
        for name, o_val in (("S", S.numpy()), ("Sh", Sh.numpy()), ("R", R.numpy()), ("final", final),
                            ("T_final", Tf.numpy())):
            worst[name] = max(worst.get(name, 0.0), float(np.abs(o_val - gpu[name]).max()))
    print(f"camera patches: {worst}; flagged decisions {flagged}, flipped {flipped}; bound-flagged px "
          f"{n_bound}/512")
    for name, e in worst.items():
        assert e <= TOL, (name, e)


def test_fluffy_banded_den_equals_tile_sum(run):
    """GPU self-consistency of the banded denominator: banded needles whose
    light bounding boxes do not overlap, rendered together, shadow nothing
    else, so each one's numerator (the tile walk, which tests every pixel of
    every tile the needle is binned to) sums exactly the beta of the pixels
    its denominator (the band-culled walk) must sum. num = den up to float32
    summation order."""
    from paper_2410_11419_amd import gs3
    sc, light, prl, op, k = run["sc"], run["light"], run["prl"], run["op"], run["k"]
    ix, iy, rx, ry = O.splat_extent(prl, op, k)
    x0, x1, y0, y1, empty = O.tile_rects(ix, iy, rx, ry, light.width, light.height)
    tiles = (x1 - x0 + 1) * (y1 - y0 + 1)
    con = prl["conic"].numpy()
    det = con[:, 0] * con[:, 2] - con[:, 1] ** 2
    banded = np.nonzero((~empty) & (tiles >= 16) & (con[:, 0] * con[:, 2] > 4 * det))[0]
    rng = np.random.default_rng(5)
    cand = np.concatenate([rng.choice(banded, 300, replace=False), rng.choice(banded, 3000, replace=False)])
    occupied = np.zeros(((light.height + 15) // 16, (light.width + 15) // 16), bool)
    chosen = []
    for j in cand:
        box = occupied[y0[j]:y1[j] + 1, x0[j]:x1[j] + 1]
        if not box.any():
            box[:] = True
            chosen.append(int(j))
    chosen = np.array(sorted(set(chosen)))
    sub = synth.subset(sc, chosen)
    ds = gs3.DeviceScene.from_host(sub)
    vb = gs3.ViewBuffer(sub.n, light.width, light.height, 1 << 24)
    gs3.gs3_preprocess(ds, light, gs3.default_consts(), gs3.GS3_DEPTH_DIST, vb)
    nd = torch.empty(2, sub.n, device="cuda")
    T = torch.empty(sub.n, device="cuda")
    gs3.gs3_shadow_splat(gs3.default_consts(), vb, nd, T)
    torch.cuda.synchronize()
    num, den = nd[0].cpu().numpy().astype(np.float64), nd[1].cpu().numpy().astype(np.float64)
    live = den > 0
    rel = np.abs(num - den)[live] / den[live]
    worst = int(np.argmax(rel))
    print(f"{len(chosen)} banded needles with disjoint light boxes: max |num - den| / den {rel.max():.2e} "
          f"(needle {chosen[live][worst]}, den {den[live][worst]:.4f}); T in [{T.min().item():.7f}, "
          f"{T.max().item():.7f}]")
    assert len(chosen) >= 40 and live.sum() >= 40
    assert rel.max() <= 1e-5
