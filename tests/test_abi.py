"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/gs3.h declares, and its host-only entry points
(constants, status strings, workspace sizing, argument validation) behave."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs3.h")
LIB = os.path.join(ROOT, "paper_2410_11419_amd", "libgs3.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs3_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["gs3_preprocess", "gs3_shadow_splat", "gs3_render", "gs3_project", "gs3_bin"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libgs3.so not built: python -m paper_2410_11419_amd.build"
    lib = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_2410_11419_amd import gs3
    assert set(declared_functions()) == set(gs3.EXPORTED)


def test_host_only_entry_points():
    from paper_2410_11419_amd import gs3
    k = gs3.default_consts()
    assert k.cutoff == pytest.approx(4.5) and k.shadow_bias == pytest.approx(0.015)
    assert k.alpha_min == pytest.approx(1 / 255) and k.alpha_max == pytest.approx(0.99)
    assert k.t_min == pytest.approx(1e-4) and k.dilation == pytest.approx(0.3)
    assert k.near_plane == pytest.approx(0.2) and k.clamp_frac == pytest.approx(1.3)
    assert gs3._lib.gs3_status_string(-3) == b"GS3_PAIR_CAPACITY_EXCEEDED"
    size = C.c_size_t()
    assert gs3._lib.gs3_view_workspace_size(1000, 128, 96, 50000, C.byref(size)) == 0
    assert size.value > 50000 * 16
    big = C.c_size_t()
    assert gs3._lib.gs3_view_workspace_size(1000, 128, 96, 100000, C.byref(big)) == 0
    assert big.value > size.value
    assert gs3._lib.gs3_view_workspace_size(-1, 128, 96, 10, C.byref(size)) == gs3.GS3_INVALID_ARG
    assert gs3._lib.gs3_view_workspace_size(10, 0, 96, 10, C.byref(size)) == gs3.GS3_INVALID_ARG
    assert b"invalid" in gs3._lib.gs3_last_error()
    # a NULL view buffer is rejected before any device work
    assert gs3._lib.gs3_view_pair_count(None, None, None) == gs3.GS3_INVALID_ARG
    vb = gs3.gs3_viewbuf(C.c_void_p(256), 10, 100, 64, 64, 1000)   # too small a workspace
    n = C.c_int64()
    assert gs3._lib.gs3_view_pair_count(C.byref(vb), C.byref(n), None) == gs3.GS3_WORKSPACE_TOO_SMALL
    vb = gs3.gs3_viewbuf(C.c_void_p(257), 1 << 30, 100, 64, 64, 1000)  # misaligned
    assert gs3._lib.gs3_view_pair_count(C.byref(vb), C.byref(n), None) == gs3.GS3_INVALID_ARG


def _status_block(generation, overflow, required):
    """A status block as the device leaves it after binning `generation`."""
    blk = (C.c_int64 * 2)()
    blk[0] = generation
    blk[1] = ((generation & 0xFFFFFF) << 40) | ((1 if overflow else 0) << 39) | required
    return blk


def test_status_block_reports_overflow_without_the_device():
    """A workspace whose status block records a completed, overflowed binning
    is refused by every call that would read its lists, before anything is
    enqueued (these calls run here without a GPU); a binning still pending
    (generation ahead of the device's word) or one within capacity is not."""
    from paper_2410_11419_amd import gs3
    size = C.c_size_t()
    assert gs3._lib.gs3_view_workspace_size(100, 64, 64, 1000, C.byref(size)) == 0
    k = gs3.default_consts()
    blk = _status_block(3, True, 12345)
    vb = gs3.gs3_viewbuf(C.c_void_p(256), size.value, 100, 64, 64, 1000, C.cast(blk, C.c_void_p))
    st, req = C.c_int32(), C.c_int64()
    assert gs3._lib.gs3_view_poll(C.byref(vb), C.byref(st), C.byref(req)) == 0
    assert (st.value, req.value) == (gs3.GS3_VIEW_OVERFLOW, 12345)
    fake = C.c_void_p(512)
    calls = {
        "gs3_shadow_splat": lambda: gs3._lib.gs3_shadow_splat(C.byref(k), C.byref(vb), fake, fake, None),
        "gs3_shadow_den": lambda: gs3._lib.gs3_shadow_den(C.byref(k), C.byref(vb), fake, None),
        "gs3_shadow_num": lambda: gs3._lib.gs3_shadow_num(C.byref(k), C.byref(vb), fake, None),
        "gs3_shadow_resolve": lambda: gs3._lib.gs3_shadow_resolve(C.byref(vb), fake, fake, None),
        "gs3_view_lists": lambda: gs3._lib.gs3_view_lists(C.byref(vb), None, None, None, None, None),
        "gs3_view_count_hits": lambda: gs3._lib.gs3_view_count_hits(C.byref(k), C.byref(vb), 0, C.c_void_p(1024),
                                                                     None),
    }
    for name, call in calls.items():
        assert call() == gs3.GS3_PAIR_CAPACITY_EXCEEDED, name
        assert b"12345" in gs3._lib.gs3_last_error(), name
    # the camera side: gs3_render is refused the same way
    cam = gs3.gs3_view()
    cam.eye[0], cam.width, cam.height, cam.fov = 4.0, 64, 64, 0.7
    scene = gs3.gs3_scene()
    scene.n, scene.k = 100, 0
    for nm in ("mean", "log_scale", "rot", "opacity_logit", "shade_rot", "albedo", "feat"):
        setattr(scene, nm, 512)
    lp = gs3.gs3_view()
    lp.eye[1], lp.width, lp.height, lp.fov = 4.0, 64, 64, 0.7
    im = gs3.gs3_images(*([512] * 7))
    assert gs3._lib.gs3_render(C.byref(scene), C.byref(cam), C.byref(lp), C.byref(k), fake, None, None, C.byref(vb),
                               C.byref(im), None) == gs3.GS3_PAIR_CAPACITY_EXCEEDED
    # a newer binning that has not finished yet: nothing is known, nothing refused
    blk[0] = 4
    assert gs3._lib.gs3_view_poll(C.byref(vb), C.byref(st), C.byref(req)) == 0
    assert (st.value, req.value) == (gs3.GS3_VIEW_PENDING, -1)
    # a binning within capacity
    ok = _status_block(7, False, 999)
    vb.status = C.cast(ok, C.c_void_p)
    assert gs3._lib.gs3_view_poll(C.byref(vb), C.byref(st), C.byref(req)) == 0
    assert (st.value, req.value) == (gs3.GS3_VIEW_OK, 999)
    # never binned
    fresh = (C.c_int64 * 2)()
    vb.status = C.cast(fresh, C.c_void_p)
    assert gs3._lib.gs3_view_poll(C.byref(vb), C.byref(st), C.byref(req)) == 0
    assert st.value == gs3.GS3_VIEW_PENDING
    vb.status = None
    assert gs3._lib.gs3_view_poll(C.byref(vb), C.byref(st), C.byref(req)) == gs3.GS3_INVALID_ARG


def test_loss_and_gradient_set_argument_checks():
    from paper_2410_11419_amd import gs3
    size = C.c_size_t()
    assert gs3._lib.gs3_l1_loss_workspace_size(0, C.byref(size)) == 0 and size.value >= 8
    assert gs3._lib.gs3_l1_loss_workspace_size(3 * 800 * 800, C.byref(size)) == 0
    assert size.value >= 8 * ((3 * 800 * 800 + 8191) // 8192) and size.value % 256 == 0
    assert gs3._lib.gs3_l1_loss_workspace_size(-1, C.byref(size)) == gs3.GS3_INVALID_ARG
    p = C.c_void_p(256)
    assert gs3._lib.gs3_l1_loss(None, p, 10, 1.0, p, None, p, 1 << 20, None) == gs3.GS3_INVALID_ARG
    assert gs3._lib.gs3_l1_loss(p, p, -1, 1.0, p, None, p, 1 << 20, None) == gs3.GS3_INVALID_ARG
    assert gs3._lib.gs3_l1_loss(p, p, 10, 1.0, p, None, C.c_void_p(260), 1 << 20, None) == gs3.GS3_INVALID_ARG
    assert gs3._lib.gs3_l1_loss(p, p, 1 << 24, 1.0, p, None, p, 8, None) == gs3.GS3_WORKSPACE_TOO_SMALL
    assert gs3._lib.gs3_grads_clear(None, 5, None) == gs3.GS3_INVALID_ARG
    assert gs3._lib.gs3_grads_clear(p, -1, None) == gs3.GS3_INVALID_ARG
    assert gs3._lib.gs3_grads_accumulate(p, None, 5, None) == gs3.GS3_INVALID_ARG


def test_view_projection_checks():
    """Orthographic views need a positive width; unknown projections are
    refused (before any device work)."""
    from paper_2410_11419_amd import gs3
    size = C.c_size_t()
    assert gs3._lib.gs3_view_workspace_size(10, 64, 64, 1000, C.byref(size)) == 0
    vb = gs3.gs3_viewbuf(C.c_void_p(256), size.value, 10, 64, 64, 1000, None)
    scene = gs3.gs3_scene()
    scene.n, scene.k = 10, 0
    for nm in ("mean", "log_scale", "rot", "opacity_logit"):
        setattr(scene, nm, 512)
    k = gs3.default_consts()
    v = gs3.gs3_view()
    v.eye[2], v.width, v.height = 4.0, 64, 64
    v.projection, v.ortho_width = gs3.GS3_ORTHOGRAPHIC, 0.0
    assert gs3._lib.gs3_project(C.byref(scene), C.byref(v), C.byref(k), 1, C.byref(vb), None) == gs3.GS3_INVALID_ARG
    assert b"ortho_width" in gs3._lib.gs3_last_error()
    v.projection = 7
    assert gs3._lib.gs3_project(C.byref(scene), C.byref(v), C.byref(k), 1, C.byref(vb), None) == gs3.GS3_INVALID_ARG


def test_preprocess_views_checks():
    """gs3_preprocess_views checks every view before enqueuing anything:
    n_views >= 1, matching sizes, and workspaces that do not overlap."""
    from paper_2410_11419_amd import gs3
    size = C.c_size_t()
    assert gs3._lib.gs3_view_workspace_size(10, 64, 64, 1000, C.byref(size)) == 0
    a = gs3.gs3_viewbuf(C.c_void_p(1 << 20), size.value, 10, 64, 64, 1000, None)
    b = gs3.gs3_viewbuf(C.c_void_p((1 << 20) + 256), size.value, 10, 64, 64, 1000, None)   # overlaps a
    scene = gs3.gs3_scene()
    scene.n, scene.k = 10, 0
    for nm in ("mean", "log_scale", "rot", "opacity_logit"):
        setattr(scene, nm, 512)
    k = gs3.default_consts()
    v = gs3.gs3_view()
    v.eye[2], v.width, v.height, v.fov = 4.0, 64, 64, 0.7
    views = (gs3.gs3_view * 2)(v, v)
    modes = (C.c_int32 * 2)(0, 1)
    vbs = (gs3.gs3_viewbuf * 2)(a, b)
    f = gs3._lib.gs3_preprocess_views
    assert f(C.byref(scene), views, modes, 0, C.byref(k), vbs, None) == gs3.GS3_INVALID_ARG
    assert f(C.byref(scene), views, modes, 2, C.byref(k), vbs, None) == gs3.GS3_INVALID_ARG
    assert b"share workspace" in gs3._lib.gs3_last_error()
    v2 = gs3.gs3_view()
    v2.eye[2], v2.width, v2.height, v2.fov = 4.0, 32, 64, 0.7
    views2 = (gs3.gs3_view * 2)(v, v2)
    b2 = gs3.gs3_viewbuf(C.c_void_p(1 << 30), size.value, 10, 64, 64, 1000, None)
    vbs2 = (gs3.gs3_viewbuf * 2)(a, b2)
    assert f(C.byref(scene), views2, modes, 2, C.byref(k), vbs2, None) == gs3.GS3_INVALID_ARG
    assert b"does not match" in gs3._lib.gs3_last_error()
    modes_bad = (C.c_int32 * 2)(0, 5)
    assert f(C.byref(scene), views, modes_bad, 2, C.byref(k), vbs2, None) == gs3.GS3_INVALID_ARG


def test_view_array_and_appearance_checks():
    """The view-array calls and the appearance model are validated on the
    host before anything reaches the device."""
    from paper_2410_11419_amd import gs3
    k = gs3.default_consts()
    L = gs3._lib
    vb = gs3.gs3_viewbuf(C.c_void_p(256), 1 << 30, 100, 64, 64, 1000)
    arr = (C.c_void_p * 1)(C.c_void_p(512))
    vbs = (gs3.gs3_viewbuf * 1)(vb)
    # no views, NULL arrays
    assert L.gs3_shadow_splat_views(C.byref(k), vbs, 0, arr, arr, None) == gs3.GS3_INVALID_ARG
    assert L.gs3_shadow_splat_views(C.byref(k), None, 1, arr, arr, None) == gs3.GS3_INVALID_ARG
    # two views sharing one workspace
    vbs2 = (gs3.gs3_viewbuf * 2)(vb, vb)
    arr2 = (C.c_void_p * 2)(C.c_void_p(512), C.c_void_p(1024))
    assert L.gs3_shadow_splat_views(C.byref(k), vbs2, 2, arr2, arr2, None) == gs3.GS3_INVALID_ARG
    assert b"share workspace memory" in L.gs3_last_error()
    # render views: a scene with an unknown appearance model is refused
    sc = gs3.gs3_scene()
    sc.n, sc.k, sc.appearance = 100, 2, 7
    for name in ("mean", "log_scale", "rot", "opacity_logit", "shade_rot", "albedo"):
        setattr(sc, name, C.c_void_p(4096))
    cam = gs3.make_view(type("V", (), dict(eye=(0.0, 0.0, 4.0), target=(0.0, 0.0, 0.0), width=64, height=64,
                                            fov=0.7, projection="perspective", ortho_width=0.0))())
    cams = (gs3.gs3_view * 1)(cam)
    ims = (gs3.gs3_images * 1)(gs3.gs3_images())
    assert L.gs3_render_views(C.byref(sc), cams, cams, 1, C.byref(k), arr, None, None, vbs, ims,
                              None) == gs3.GS3_INVALID_ARG
    assert b"appearance" in L.gs3_last_error()
    # the basis model needs its own pointers
    sc.appearance = gs3.GS3_APPEARANCE_BASIS
    assert L.gs3_render_views(C.byref(sc), cams, cams, 1, C.byref(k), arr, None, None, vbs, ims,
                              None) == gs3.GS3_INVALID_ARG
    assert b"basis" in L.gs3_last_error()
    # backward workspace per appearance: the basis model keeps more per Gaussian
    a, b = C.c_size_t(), C.c_size_t()
    assert L.gs3_backward_workspace_size_for(gs3.GS3_APPEARANCE_LOBES, 300000, 1024, 1024, C.byref(a)) == 0
    assert L.gs3_backward_workspace_size_for(gs3.GS3_APPEARANCE_BASIS, 300000, 1024, 1024, C.byref(b)) == 0
    # lobes model: per Gaussian the gradient staging (6 + 7 + 6 + 2 floats),
    # each MLP's input and output-layer gradient (17 + 1 + 22 + 3 rows)
    assert b.value > a.value > 300000 * (21 + 43) * 4
    assert L.gs3_backward_workspace_size_for(5, 10, 8, 8, C.byref(a)) == gs3.GS3_INVALID_ARG
