"""GPU tests of the batched entry points: several views in one launch
sequence give exactly (bit for bit) the splats and tile lists of the same
views preprocessed one at a time, across batch chunks, mixed sizes, tile
pass counts, packed and two-array pair sorts, and a view that overflows."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2410_11419_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs3():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2410_11419_amd import gs3 as g
    assert g.device_ok(), "libgs3 needs a gfx950 device"
    return g


def _views():
    rng = np.random.default_rng(17)
    v = []
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 128, 128, 40.0), "z"))
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 128, 128, 60.0), "dist"))
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 200, 152, 40.0), "z"))     # ragged tiles
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 1, 1, 40.0), "z"))         # one pixel
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 3, 5, 60.0), "dist"))      # one tile
    v.append((synth.make_directional(rng.standard_normal(3), 160, 160, 3.6), "dist"))  # orthographic
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 1024, 1024, 40.0), "dist"))  # two tile passes
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 64, 48, 40.0), "z"))
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 800, 600, 50.0), "z"))      # second chunk
    # 1M tiles (20 bits) + 13 id bits: the two-array sort, three tile passes
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 16384, 16384, 40.0), "z"))
    v.append((synth.make_view(rng.standard_normal(3), 4.0, 96, 256, 30.0), "dist"))
    return v


def _mode(g, m):
    return g.GS3_DEPTH_Z if m == "z" else g.GS3_DEPTH_DIST


def _single(g, ds, view, mode, consts):
    cap = 1 << 16
    while True:
        vb = g.ViewBuffer(ds.n, view.width, view.height, cap)
        g.gs3_preprocess(ds, view, consts, mode, vb)
        try:
            return vb, g.gs3_view_pair_count(vb)
        except g.Gs3Error as e:
            assert e.status == g.GS3_PAIR_CAPACITY_EXCEEDED
            cap = e.required + 1000


def _export(g, vb):
    lists = [t.cpu().numpy() for t in g.gs3_view_lists(vb)]
    splats = [t.cpu().numpy() for t in g.gs3_view_splats(vb)]
    return lists, splats


def test_preprocess_views_equals_single(gs3):
    sc, _, _ = synth.scene_small(seed=6)
    ds = gs3.DeviceScene.from_host(sc)
    k = gs3.default_consts()
    views = _views()
    singles, caps = [], []
    for view, m in views:
        vb, p = _single(gs3, ds, view, _mode(gs3, m), k)
        singles.append(_export(gs3, vb))
        caps.append(p + 7)
    packed = [vb_bits for vb_bits in (math.ceil(math.log2(max(2, ((v.width + 15) // 16) * ((v.height + 15) // 16))))
                                      for v, _ in views)]
    print(f"{len(views)} views, pair counts {[c - 7 for c in caps]}, tile bits {packed}")
    vbs = [gs3.ViewBuffer(ds.n, v.width, v.height, c) for (v, _), c in zip(views, caps)]
    gs3.gs3_preprocess_views(ds, [v for v, _ in views], [_mode(gs3, m) for _, m in views], k, vbs)
    for i, vb in enumerate(vbs):
        assert gs3.gs3_view_pair_count(vb) == caps[i] - 7
        (ts, te, ids, keys), splats = _export(gs3, vb)
        (ts0, te0, ids0, keys0), splats0 = singles[i]
        np.testing.assert_array_equal(te - ts, te0 - ts0)
        np.testing.assert_array_equal(ids, ids0)
        np.testing.assert_array_equal(keys, keys0)
        for a, b in zip(splats, splats0):
            np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
    # the oracle's brute-force binning of two of them, from the GPU's extents
    for i in (2, 9):
        view = views[i][0]
        (ts, te, ids, keys), (_, _, _, depth, ext) = singles[i]
        ext = ext.astype(np.int64)
        counts, oids, okeys = O.bin_tiles(ext[0], ext[1], ext[2], ext[3], depth, view.width, view.height)
        np.testing.assert_array_equal(te - ts, counts)
        np.testing.assert_array_equal(ids, oids)
        np.testing.assert_array_equal(keys.view(np.uint64), okeys)


def test_preprocess_views_overflow_is_per_view(gs3):
    sc, _, _ = synth.scene_small(seed=7)
    ds = gs3.DeviceScene.from_host(sc)
    k = gs3.default_consts()
    views = _views()[:4]
    ref = [_single(gs3, ds, v, _mode(gs3, m), k) for v, m in views]
    caps = [p + 3 for _, p in ref]
    caps[1] = ref[1][1] // 3          # too small: overflows
    vbs = [gs3.ViewBuffer(ds.n, v.width, v.height, c) for (v, _), c in zip(views, caps)]
    gs3.gs3_preprocess_views(ds, [v for v, _ in views], [_mode(gs3, m) for _, m in views], k, vbs)
    for i, vb in enumerate(vbs):
        if i == 1:
            with pytest.raises(gs3.Gs3Error) as ei:
                gs3.gs3_view_pair_count(vb)
            assert ei.value.status == gs3.GS3_PAIR_CAPACITY_EXCEEDED and ei.value.required == ref[1][1]
            state, req = gs3.gs3_view_poll(vb)
            assert state == gs3.GS3_VIEW_OVERFLOW and req == ref[1][1]
        else:
            assert gs3.gs3_view_pair_count(vb) == ref[i][1]
            np.testing.assert_array_equal(gs3.gs3_view_lists(vb)[2].cpu().numpy(),
                                          gs3.gs3_view_lists(ref[i][0])[2].cpu().numpy())


@pytest.mark.parametrize("overlap", [False, True])
def test_renderer_batched_views(gs3, overlap):
    """Renderer(batch_views=True) preprocesses the light and camera views in
    one launch sequence; frames equal the unbatched renderer's (the shadow
    numerator's float atomics may add in another order: 1e-6)."""
    sc = synth.make_scene(20000, 8, seed=8, means="shell", mlps=True)
    ds = gs3.DeviceScene.from_host(sc)
    a = gs3.Renderer(ds)
    b = gs3.Renderer(ds, batch_views=True)
    rng = np.random.default_rng(4)
    for _ in range(3):
        cam = synth.make_view(rng.standard_normal(3), 4.0, 160, 120, 40.0)
        light = synth.make_view(rng.standard_normal(3), 4.0, 192, 192, 40.0)
        ra = a.render(cam, light, check=True)
        b.render(cam, light, check=True)
        rb = b.render(cam, light, check=False, overlap=overlap)
        torch.cuda.synchronize()
        assert not b.overflowed()
        for key in ("final", "T_final", "S"):
            assert float((ra[key] - rb[key]).abs().max()) <= 1e-6, key
        assert float((ra["T"] - rb["T"]).abs().max()) <= 1e-6


def _requests(n, seed, sizes, light_sizes):
    rng = np.random.default_rng(seed)
    cams, lights = [], []
    for i in range(n):
        w, h = sizes[i % len(sizes)]
        cams.append(synth.make_view(rng.standard_normal(3), 4.0, w, h, 40.0))
        lw, lh = light_sizes[i % len(light_sizes)]
        if lw < 0:
            lights.append(synth.make_directional(rng.standard_normal(3), -lw, -lh, 2.4))
        else:
            lights.append(synth.make_view(rng.standard_normal(3), 4.0, lw, lh, 60.0))
    return cams, lights


@pytest.mark.parametrize("appearance", ["lobes", "basis"])
def test_render_batched_equals_single(gs3, appearance):
    """gs3_preprocess_views + gs3_shadow_splat_views + gs3_render_views over
    eleven requests of mixed camera and light sizes (two launch chunks, a
    directional light, a light shared by two requests, a one-tile camera)
    against each request rendered alone: shadow values and every image
    within 1e-5 (the shadow numerator's float atomics may add in another
    order), integer contribution counts equal."""
    if appearance == "lobes":
        sc = synth.make_scene(6000, 4, seed=21, means="shell", mlps=True, log_scale_mu=(-3.6,) * 3)
    else:
        sc = synth.make_basis_scene(6000, 21, means="shell", mlps=True, log_scale_mu=(-3.6,) * 3)
    ds = gs3.DeviceScene.from_host(sc)
    sizes = [(128, 128), (200, 152), (96, 64), (16, 16), (256, 256), (72, 200)]
    lsizes = [(128, 128), (-160, -160), (200, 200), (64, 64)]
    cams, lights = _requests(11, 31, sizes, lsizes)
    lights[7] = lights[2]                         # a shared light
    rnds = [gs3.Renderer(ds) for _ in cams]
    outs = gs3.render_batched(rnds, cams, lights)
    got = [{k: v.clone() for k, v in o.items()} for o in outs]
    torch.cuda.synchronize()
    assert not any(r.overflowed() for r in rnds)
    single = gs3.Renderer(ds)
    worst_T = worst_im = 0.0
    for i, (cam, light) in enumerate(zip(cams, lights)):
        ref = single.render(cam, light, overlap=False)
        worst_T = max(worst_T, float((got[i]["T"][:sc.n] - ref["T"][:sc.n]).abs().max()))
        for k in ("final", "S", "Sh", "R", "T_final", "colour"):
            worst_im = max(worst_im, float((got[i][k] - ref[k]).abs().max()))
        assert torch.equal(got[i]["n_contrib"], ref["n_contrib"]) or \
            float((got[i]["n_contrib"] != ref["n_contrib"]).float().mean()) < 1e-3
    print(f"[{appearance}] batched vs single: T {worst_T:.2e}, images {worst_im:.2e}")
    assert worst_T <= 1e-5 and worst_im <= 1e-5


def test_batched_entry_points_check_arguments(gs3):
    sc = synth.make_scene(500, 2, seed=3, means="cube")
    ds = gs3.DeviceScene.from_host(sc)
    rnd = gs3.Renderer(ds)
    cam, light = _requests(1, 5, [(64, 64)], [(64, 64)])
    out = rnd.render(cam[0], light[0])
    lvb = rnd.vbs[("light", 64, 64)]
    with pytest.raises(gs3.Gs3Error):
        gs3.gs3_shadow_splat_views(rnd.consts, [lvb, lvb], [rnd.num_den, rnd.num_den], [rnd.T, rnd.T])  # shared ws
    cvb = rnd.vbs[("cam", 64, 64)]
    im = rnd._images(64, 64)
    with pytest.raises(gs3.Gs3Error):   # a light view in place of a camera buffer of the wrong size
        gs3.gs3_render_views(ds, [cam[0]], [light[0]], rnd.consts, [rnd.T],
                             [gs3.ViewBuffer(ds.n, 32, 32, 1 << 16)], [im])
    gs3.gs3_render_views(ds, [cam[0]], [light[0]], rnd.consts, [out["T"]], [cvb], [im])
    torch.cuda.synchronize()
