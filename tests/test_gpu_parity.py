"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Integer work (tile keys, counts, sorted lists) must match bit for bit;
floating-point outputs (projection, shadow values, per-Gaussian colours,
images) must match within 1e-4 max abs everywhere. Threshold decisions that
float32 rounding may take either way are flagged by the oracle; the GPU's
outcome of each is found and the oracle rendered with it
(tests/parity_resolve.py), so no output is left out."""
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


@pytest.fixture(scope="module")
def gs3():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2410_11419_amd import gs3 as g
    assert g.device_ok(), "libgs3 needs a gfx950 device"
    return g


def _view(eye, w, h, fov=40.0):
    return synth.View(eye=np.asarray(eye, np.float64), target=np.zeros(3), width=w, height=h,
                      fov=math.radians(fov))


# ------------------------------------------------------------- binning

def _random_extents(rng, n, W, H, max_r=40, cull_frac=0.1, ties=True):
    ix = rng.integers(-60, W + 60, n).astype(np.int32)
    iy = rng.integers(-60, H + 60, n).astype(np.int32)
    rx = rng.integers(1, max_r, n).astype(np.int32)
    ry = rng.integers(1, max_r, n).astype(np.int32)
    cull = rng.random(n) < cull_frac
    rx[cull] = -1
    ry[cull & (rng.random(n) < 0.5)] = 0
    depth = rng.uniform(0.5, 8.0, n).astype(np.float32)
    if ties and n > 10:
        depth[rng.integers(0, n, n // 10)] = depth[0]     # many exact ties
    return ix, iy, rx, ry, depth


def _bin_gpu(g, ix, iy, rx, ry, depth, W, H, capacity):
    n = len(ix)
    vb = g.ViewBuffer(n, W, H, capacity)
    dev = [torch.as_tensor(a).cuda() for a in (ix, iy, rx, ry, depth)]
    if n == 0:
        dev = [torch.zeros(1, dtype=a.dtype).cuda() for a in dev]
    g.gs3_bin(*dev, vb)
    return vb


@pytest.mark.parametrize("case", [
    dict(n=10000, W=256, H=256, seed=1),           # 256 tiles: one tile pass
    dict(n=30000, W=1000, H=600, seed=2),          # 2,394 tiles (ragged edge): two passes
    dict(n=5000, W=10, H=7, seed=3, max_r=4),      # one tile: no tile pass
    dict(n=4097, W=300, H=200, seed=4, cull_frac=1.0),   # everything culled
    dict(n=1, W=64, H=64, seed=5),
    # 21 id bits + 12 tile bits do not pack into one word: the two-array sort
    dict(n=(1 << 20) + 5, W=1024, H=768, seed=6, max_r=3),
    # the largest view whose pair offsets are formed inside the emission
    # (2^19 splats), and one splat more (separate scan launches)
    dict(n=128 * 4096, W=512, H=384, seed=7, max_r=5),
    dict(n=128 * 4096 + 1, W=512, H=384, seed=8, max_r=5),
])
def test_binning_bit_exact(gs3, case):
    rng = np.random.default_rng(case["seed"])
    W, H = case["W"], case["H"]
    ix, iy, rx, ry, depth = _random_extents(rng, case["n"], W, H, case.get("max_r", 40),
                                            case.get("cull_frac", 0.1))
    counts, ids, keys = O.bin_tiles(ix, iy, rx, ry, depth, W, H)
    P = int(counts.sum())
    vb = _bin_gpu(gs3, ix, iy, rx, ry, depth, W, H, capacity=P + 17)
    assert gs3.gs3_view_pair_count(vb) == P
    ts, te, gids, gkeys = gs3.gs3_view_lists(vb)
    ts, te = ts.cpu().numpy(), te.cpu().numpy()
    np.testing.assert_array_equal(te - ts, counts)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    nz = counts > 0
    np.testing.assert_array_equal(ts[nz], starts[nz])
    np.testing.assert_array_equal(gids.cpu().numpy(), ids)
    np.testing.assert_array_equal(gkeys.cpu().numpy().view(np.uint64), keys)
    # run twice: identical lists
    vb2 = _bin_gpu(gs3, ix, iy, rx, ry, depth, W, H, capacity=P + 17)
    np.testing.assert_array_equal(gs3.gs3_view_lists(vb2)[2].cpu().numpy(), ids)


def test_binning_empty_and_overflow(gs3):
    vb = _bin_gpu(gs3, *[np.zeros(0, t) for t in (np.int32,) * 4 + (np.float32,)], 64, 64, capacity=8)
    assert gs3.gs3_view_pair_count(vb) == 0
    ts, te, ids, keys = gs3.gs3_view_lists(vb)
    assert (te - ts).sum().item() == 0
    rng = np.random.default_rng(9)
    ix, iy, rx, ry, depth = _random_extents(rng, 2000, 128, 128)
    counts, _, _ = O.bin_tiles(ix, iy, rx, ry, depth, 128, 128)
    vb = _bin_gpu(gs3, ix, iy, rx, ry, depth, 128, 128, capacity=int(counts.sum()) // 2)
    with pytest.raises(gs3.Gs3Error) as ei:
        gs3.gs3_view_pair_count(vb)
    assert ei.value.status == gs3.GS3_PAIR_CAPACITY_EXCEEDED
    assert ei.value.required == int(counts.sum())


# ---------------------------------------------------------- projection

@pytest.mark.parametrize("mode", ["z", "dist"])
def test_projection_parity(gs3, mode):
    sc, cam, light = synth.scene_small()
    view = cam if mode == "z" else light
    ds = gs3.DeviceScene.from_host(sc)
    vb = gs3.ViewBuffer(sc.n, view.width, view.height, 1 << 18)
    gs3.gs3_project(ds, view, gs3.default_consts(), gs3.GS3_DEPTH_Z if mode == "z" else gs3.GS3_DEPTH_DIST, vb)
    mean2d, conic, opac, depth, ext = [t.cpu().numpy() for t in gs3.gs3_view_splats(vb)]
    p = O.scene_tensors(sc)
    cov = O.covariance(p["log_scale"], p["rot"])
    pr = O.project(p["mean"], cov, view, O.Consts(), mode)
    op = O.sigmoid(p["opacity_logit"])
    ix, iy, rx, ry = O.splat_extent(pr, op, O.Consts())
    live = rx > 0
    # the GPU also culls splats whose rectangle misses the image
    x0, x1, y0, y1, empty = O.tile_rects(ix, iy, rx, ry, view.width, view.height)
    live = live & ~empty
    assert live.sum() > 1000
    np.testing.assert_array_equal(ext[2] > 0, live)
    np.testing.assert_allclose(mean2d[0][live], pr["u"].numpy()[live], atol=2e-5, rtol=0)
    np.testing.assert_allclose(mean2d[1][live], pr["v"].numpy()[live], atol=2e-5, rtol=0)
    ref_con = pr["conic"].numpy()[live].T
    np.testing.assert_allclose(conic[:, live], ref_con, rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(opac[live], op.detach().numpy()[live], rtol=2e-7)
    np.testing.assert_allclose(depth[live], pr["depth"].numpy()[live], rtol=2e-7)
    np.testing.assert_array_equal(ext[0][live], ix[live])
    np.testing.assert_array_equal(ext[1][live], iy[live])
    # extents are ceil() of an exact value: equal unless that value sits on an integer
    assert (np.abs(ext[2][live] - rx[live]) <= 1).all() and (np.abs(ext[3][live] - ry[live]) <= 1).all()
    assert (ext[2][live] != rx[live]).mean() < 1e-3


# -------------------------------------------------------- full forward

def _gpu_px(out, npx):
    return {k: out[k].cpu().numpy().reshape(-1, npx).squeeze(0) if out[k].dim() == 2 else
            out[k].cpu().numpy().reshape(3, npx) for k in ("final", "S", "Sh", "R", "T_final")}


def _compare_render(g, sc, cam, light, consts_o, consts_g, use_mlps, tag, nonempty=True):
    """Every output of the GPU render against the oracle whose float32-
    ambiguous threshold decisions follow the GPU's (tests/parity_resolve.py):
    shadow values, per-Gaussian colours, T', r and every pixel of every
    image, with nothing left out. Also reports how many outputs the oracle's
    error bound alone would have left out and their error after resolution."""
    ds = g.DeviceScene.from_host(sc)
    rnd = g.Renderer(ds, consts_g, use_mlps=use_mlps)
    out = rnd.render(cam, light)
    torch.cuda.synchronize()
    phi = sc.phi.layers if (use_mlps and sc.phi) else None
    psi = sc.psi.layers if (use_mlps and sc.psi) else None
    T_g = out["T"].cpu().numpy()[:sc.n]
    px = _gpu_px(out, cam.width * cam.height)
    ref, info = resolve(sc, cam, light, consts_o, phi, psi, T_g, px)
    im = O.render_images(ref, cam)
    T_o = ref["T"].detach().numpy()
    errT_all = np.abs(T_g - T_o)
    # per-Gaussian colours (c, T', r)
    col = out["colour"].cpu().numpy()[:, :sc.n]
    c_o = ref["c"].detach().numpy().T
    r_o = ref["r"].detach().numpy().T
    tp_o = ref["Tp"].detach().numpy()
    err_c = np.abs(col[0:3] - c_o).max() if sc.n else 0.0
    err_r = (np.abs(col[4:7] - r_o).max() if use_mlps else np.abs(col[4:7]).max()) if sc.n else 0.0
    err_tp = np.abs(col[3] - tp_o).max() if sc.n else 0.0
    errT = errT_all.max() if sc.n else 0.0
    # images: every pixel
    errs, img_err = {}, None
    for key in ("final", "S", "Sh", "R", "T_final"):
        d = np.abs(out[key].cpu().numpy() - im[key])
        errs[key] = float(d.max())
        dd = d if d.ndim == 2 else d.max(0)
        img_err = dd if img_err is None else np.maximum(img_err, dd)
    # what the bound-based mask alone would have left out, and its error now
    bmT = ref["amb_T"].numpy() > AMB_BUDGET
    bmP = im["amb_px"] > AMB_BUDGET
    mT = float(errT_all[bmT].max()) if bmT.any() else 0.0
    mP = float(img_err[bmP].max()) if bmP.any() else 0.0
    print(f"[{tag}] T err {errT:.2e}, c {err_c:.2e}, T' {err_tp:.2e}, r {err_r:.2e}, images {errs}; "
          f"{describe(info)}; bound-flagged T {int(bmT.sum())}/{sc.n} (max err {mT:.2e}, "
          f"{int((errT_all[bmT] > TOL).sum())} above {TOL}), bound-flagged px {int(bmP.sum())}/{bmP.size} "
          f"(max err {mP:.2e}, {int((img_err[bmP] > TOL).sum())} above {TOL})")
    assert not info["unresolved_T"].any() and not info["unresolved_px"].any()
    assert errT <= TOL
    assert err_c <= TOL and err_tp <= TOL and err_r <= TOL
    for key, v in errs.items():
        assert v <= TOL, (key, v)
    if nonempty:    # the images are not trivially empty
        assert (im["T_final"] < 0.5).mean() > 0.05
    return out, ref


def test_render_parity_small_scene(gs3):
    sc, cam, light = synth.scene_small()
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), False, "small")


def test_render_parity_with_mlps_ragged(gs3):
    sc = synth.make_scene(12000, 8, seed=5, means="shell", mlps=True, log_scale_mu=(-3.6,) * 3)
    rng = np.random.default_rng(1)
    cam = synth.make_view(rng.standard_normal(3), 4.0, 200, 152, 40.0)     # ragged tiles
    light = synth.make_view(rng.standard_normal(3), 4.0, 240, 240, 40.0)
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "mlp")


@pytest.mark.parametrize("scale", [1e-3, 1e3])
def test_render_parity_mlp_activation_scale(gs3, scale):
    # The MLP hidden layers run as split half-precision products. Scaling the
    # first layer's weights and every hidden bias by s and the output layer's
    # weights by 1/s leaves the network's function unchanged (ReLU is
    # positively homogeneous) while the hidden activations become s times
    # their usual size: the split must hold its accuracy over that range.
    sc = synth.make_scene(4096, 4, seed=11, means="shell", mlps=True, log_scale_mu=(-3.6,) * 3)
    for mlp in (sc.phi, sc.psi):
        L = mlp.layers
        L[0] = ((L[0][0] * scale).astype(np.float32), (L[0][1] * scale).astype(np.float32))
        L[1] = (L[1][0], (L[1][1] * scale).astype(np.float32))
        L[2] = (L[2][0], (L[2][1] * scale).astype(np.float32))
        L[3] = ((L[3][0] / scale).astype(np.float32), L[3][1])
    rng = np.random.default_rng(2)
    cam = synth.make_view(rng.standard_normal(3), 4.0, 128, 128, 40.0)
    light = synth.make_view(rng.standard_normal(3), 4.0, 128, 128, 60.0)
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, f"mlp_scale_{scale:g}")


def test_render_parity_ragged_light(gs3):
    # a light view whose size is not a multiple of the 16-px tile in either
    # direction: the shadow kernels' partial last tile column and row (lane
    # masks in the denominator, bounds checks in the numerator)
    sc, cam, _ = synth.scene_small(seed=2)
    rng = np.random.default_rng(21)
    light = synth.make_view(rng.standard_normal(3), 4.0, 184, 136, 50.0)
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), False, "ragged_light")


def banded_count(sc, light):
    """Splats of the light view on the denominator's banded path: 16 tiles
    or more, bounding box over 2.5x the ellipse (conic a c > 4 det)."""
    p = O.scene_tensors(sc)
    cov = O.covariance(p["log_scale"], p["rot"])
    op = O.sigmoid(p["opacity_logit"])
    pr = O.project(p["mean"], cov, light, O.Consts(), "dist")
    ix, iy, rx, ry = O.splat_extent(pr, op, O.Consts())
    x0, x1, y0, y1, empty = O.tile_rects(ix, iy, rx, ry, light.width, light.height)
    con = pr["conic"].numpy()
    det = con[:, 0] * con[:, 2] - con[:, 1] ** 2
    return int(((~empty) & ((x1 - x0 + 1) * (y1 - y0 + 1) >= 16) & (con[:, 0] * con[:, 2] > 4 * det)).sum())


def test_render_parity_banded_needles(gs3):
    # long thin needles whose light footprints take the denominator's banded
    # path (per tile row only the ellipse's own x-band is evaluated)
    sc, cam, light = synth.scene_needles(seed=0)
    nb = banded_count(sc, light)
    print(f"[needles] {nb} banded splats in the light view")
    assert nb >= 10
    _compare_render(gs3, sc, cam, light, O.Consts(), gs3.default_consts(), True, "needles")


def test_render_parity_bias_and_stop_variants(gs3):
    sc, cam, light = synth.scene_small(seed=3)
    ko = O.Consts(shadow_bias=0.05, t_min=0.01, alpha_max=0.9)
    kg = gs3.make_consts(shadow_bias=0.05, t_min=0.01, alpha_max=0.9)
    _compare_render(gs3, sc, cam, light, ko, kg, False, "variant")


def test_render_smooth_mode(gs3):
    sc, cam, light = synth.scene_gradcheck(seed=4, n=200)
    kg = gs3.make_consts(dilation=0.0, cutoff=math.inf, alpha_min=0.0, alpha_max=1.0, t_min=0.0,
                         shadow_bias=0.0)
    _compare_render(gs3, sc, cam, light, O.SMOOTH, kg, True, "smooth")


def test_render_edge_cases(gs3):
    # empty scene
    sc, cam, light = synth.scene_small()
    empty = synth.subset(sc, np.zeros(0, np.int64))
    ds = gs3.DeviceScene.from_host(empty)
    out = gs3.Renderer(ds, use_mlps=False).render(cam, light)
    assert (out["T_final"] == 1).all() and (out["final"] == 0).all()
    # every Gaussian behind the camera
    back = synth.subset(sc, np.arange(300))
    back.mean = (back.mean * 0.1 + 1.5 * cam.eye[:, None]).astype(np.float32)   # 2 units behind the eye
    out = gs3.Renderer(gs3.DeviceScene.from_host(back), use_mlps=False).render(cam, light)
    assert (out["T_final"] == 1).all() and (out["final"] == 0).all()
    # a one-pixel camera and a tiny light view
    tiny = _view(cam.eye, 1, 1)
    small_light = _view(light.eye, 3, 5, 60)
    sub = synth.subset(sc, np.arange(500))
    _compare_render(gs3, sub, tiny, small_light, O.Consts(), gs3.default_consts(), False, "tiny",
                    nonempty=False)


def test_render_overlapped_streams_match_serial(gs3):
    # Renderer.render(overlap=True) runs the camera preprocess and the shadow
    # denominator on side streams; over consecutive frames of different views
    # it must give the serial result bit for bit (the numerator's terms are
    # summed in fixed point, so the order of its atomics does not matter)
    sc = synth.make_scene(20000, 8, seed=8, means="shell", mlps=True)
    ds = gs3.DeviceScene.from_host(sc)
    views = [(synth.make_view(np.random.default_rng(s).standard_normal(3), 4.0, 160, 120, 40.0),
              synth.make_view(np.random.default_rng(s + 50).standard_normal(3), 4.0, 192, 192, 40.0))
             for s in range(3)]
    a = gs3.Renderer(ds)
    b = gs3.Renderer(ds)
    for cam, light in views:       # size buffers, check capacity
        a.render(cam, light, check=True)
        b.render(cam, light, check=True)
    for cam, light in views * 2:
        ra = {k: v.clone() for k, v in a.render(cam, light, check=False, overlap=True).items()}
        rb = b.render(cam, light, check=False, overlap=False)
        torch.cuda.synchronize()
        for key in ("final", "S", "Sh", "R", "T_final", "T"):
            assert torch.equal(ra[key], rb[key]), key
