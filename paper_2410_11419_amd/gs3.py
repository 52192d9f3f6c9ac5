"""ctypes binding of libgs3.so (include/gs3.h).

Functions named like the C entry points marshal torch CUDA tensors into
the C structs and call the library on torch's current HIP stream; every
step of the path runs in the library's kernels. ``Renderer`` owns the view
workspaces and output tensors of a scene and chains the calls for one
relit frame.

Importing this module loads the library and raises ``ImportError`` if it has
not been built (``python -m paper_2410_11419_amd.build``); there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
from typing import Dict, Optional, Sequence

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgs3.so")

GS3_OK = 0
GS3_INVALID_ARG = -1
GS3_WORKSPACE_TOO_SMALL = -2
GS3_PAIR_CAPACITY_EXCEEDED = -3
GS3_HIP_ERROR = -4
GS3_UNSUPPORTED = -5
GS3_DEPTH_Z = 0
GS3_DEPTH_DIST = 1

EXPORTED = [
    "gs3_consts_default", "gs3_status_string", "gs3_last_error", "gs3_device_ok",
    "gs3_view_workspace_size", "gs3_project", "gs3_bin", "gs3_preprocess", "gs3_preprocess_views",
    "gs3_view_pair_count", "gs3_view_lists", "gs3_view_splats", "gs3_view_count_hits", "gs3_shadow_splat",
    "gs3_shadow_den", "gs3_shadow_num", "gs3_shadow_resolve", "gs3_render",
    "gs3_sort", "gs3_shade", "gs3_render_shaded", "gs3_backward_workspace_size", "gs3_render_backward",
    "gs3_view_poll", "gs3_l1_loss_workspace_size", "gs3_l1_loss", "gs3_grads_clear", "gs3_grads_accumulate",
    "gs3_l1_loss_noalloc", "gs3_dssim_loss_workspace_size", "gs3_dssim_loss", "gs3_adam_step",
    "gs3_image_accumulate", "gs3_backward_workspace_size_for", "gs3_shadow_splat_views", "gs3_render_views",
]
GS3_APPEARANCE_LOBES, GS3_APPEARANCE_BASIS = 0, 1
BASIS_NAMES = ("spec_albedo", "basis_weight", "latent", "basis_rot", "basis_log_sigma")
GS3_VIEW_PENDING, GS3_VIEW_OK, GS3_VIEW_OVERFLOW = 0, 1, 2


class gs3_consts(C.Structure):
    _fields_ = [("near_plane", C.c_float), ("clamp_frac", C.c_float), ("dilation", C.c_float),
                ("cutoff", C.c_float), ("alpha_min", C.c_float), ("alpha_max", C.c_float),
                ("t_min", C.c_float), ("shadow_bias", C.c_float)]


GS3_PERSPECTIVE, GS3_ORTHOGRAPHIC = 0, 1


class gs3_view(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("width", C.c_int32),
                ("height", C.c_int32), ("fov", C.c_double), ("projection", C.c_int32),
                ("ortho_width", C.c_double)]


class gs3_scene(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("log_scale", C.c_void_p), ("rot", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("shade_rot", C.c_void_p), ("albedo", C.c_void_p),
                ("lobe_axis", C.c_void_p), ("lobe_log_sharp", C.c_void_p), ("lobe_amp", C.c_void_p),
                ("feat", C.c_void_p), ("n", C.c_int64), ("k", C.c_int32), ("appearance", C.c_int32),
                ("spec_albedo", C.c_void_p), ("basis_weight", C.c_void_p), ("latent", C.c_void_p),
                ("basis_rot", C.c_void_p), ("basis_log_sigma", C.c_void_p)]


class gs3_mlp(C.Structure):
    _fields_ = [("w", C.c_void_p * 4), ("b", C.c_void_p * 4), ("n_in", C.c_int32), ("n_out", C.c_int32)]


class gs3_viewbuf(C.Structure):
    _fields_ = [("ws", C.c_void_p), ("ws_bytes", C.c_size_t), ("n", C.c_int64), ("width", C.c_int32),
                ("height", C.c_int32), ("pair_capacity", C.c_int64), ("status", C.c_void_p)]


class gs3_images(C.Structure):
    _fields_ = [("final_rgb", C.c_void_p), ("shading", C.c_void_p), ("shadow", C.c_void_p),
                ("residual", C.c_void_p), ("t_final", C.c_void_p), ("n_contrib", C.c_void_p),
                ("colour", C.c_void_p)]


class gs3_grads(C.Structure):
    _fields_ = [(nm, C.c_void_p) for nm in ("mean", "log_scale", "rot", "opacity_logit", "shade_rot", "albedo",
                                             "lobe_axis", "lobe_log_sharp", "lobe_amp", "feat")] + \
               [("phi_w", C.c_void_p * 4), ("phi_b", C.c_void_p * 4), ("psi_w", C.c_void_p * 4),
                ("psi_b", C.c_void_p * 4)] + [(nm, C.c_void_p) for nm in BASIS_NAMES]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run `python -m paper_2410_11419_amd.build`")
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    sig = {
        "gs3_consts_default": (None, [P(gs3_consts)]),
        "gs3_status_string": (C.c_char_p, [C.c_int]),
        "gs3_last_error": (C.c_char_p, []),
        "gs3_device_ok": (C.c_int, []),
        "gs3_view_workspace_size": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int64, P(C.c_size_t)]),
        "gs3_project": (C.c_int, [P(gs3_scene), P(gs3_view), P(gs3_consts), C.c_int32, P(gs3_viewbuf), C.c_void_p]),
        "gs3_bin": (C.c_int, [C.c_void_p] * 5 + [P(gs3_viewbuf), C.c_void_p]),
        "gs3_preprocess_views": (C.c_int, [P(gs3_scene), P(gs3_view), P(C.c_int32), C.c_int32, P(gs3_consts),
                                           P(gs3_viewbuf), C.c_void_p]),
        "gs3_preprocess": (C.c_int, [P(gs3_scene), P(gs3_view), P(gs3_consts), C.c_int32, P(gs3_viewbuf),
                                     C.c_void_p]),
        "gs3_view_pair_count": (C.c_int, [P(gs3_viewbuf), P(C.c_int64), C.c_void_p]),
        "gs3_view_lists": (C.c_int, [P(gs3_viewbuf)] + [C.c_void_p] * 4 + [C.c_void_p]),
        "gs3_view_splats": (C.c_int, [P(gs3_viewbuf)] + [C.c_void_p] * 5 + [C.c_void_p]),
        "gs3_view_count_hits": (C.c_int, [P(gs3_consts), P(gs3_viewbuf), C.c_int32, C.c_void_p, C.c_void_p]),
        "gs3_shadow_splat": (C.c_int, [P(gs3_consts), P(gs3_viewbuf), C.c_void_p, C.c_void_p, C.c_void_p]),
        "gs3_shadow_den": (C.c_int, [P(gs3_consts), P(gs3_viewbuf), C.c_void_p, C.c_void_p]),
        "gs3_shadow_num": (C.c_int, [P(gs3_consts), P(gs3_viewbuf), C.c_void_p, C.c_void_p]),
        "gs3_shadow_resolve": (C.c_int, [P(gs3_viewbuf), C.c_void_p, C.c_void_p, C.c_void_p]),
        "gs3_sort": (C.c_int, [P(gs3_viewbuf), C.c_void_p]),
        "gs3_shade": (C.c_int, [P(gs3_scene), P(gs3_view), P(gs3_view), P(gs3_mlp), P(gs3_viewbuf),
                                C.c_void_p, C.c_void_p]),
        "gs3_render_shaded": (C.c_int, [P(gs3_scene), P(gs3_view), P(gs3_view), P(gs3_consts), C.c_void_p,
                                        P(gs3_mlp), P(gs3_viewbuf), P(gs3_images), C.c_void_p]),
        "gs3_backward_workspace_size": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, P(C.c_size_t)]),
        "gs3_backward_workspace_size_for": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, C.c_int32, P(C.c_size_t)]),
        "gs3_render_backward": (C.c_int, [P(gs3_scene), P(gs3_view), P(gs3_view), P(gs3_consts), C.c_void_p,
                                          C.c_void_p, P(gs3_mlp), P(gs3_mlp), P(gs3_viewbuf), P(gs3_viewbuf),
                                          P(gs3_images), C.c_void_p, P(gs3_grads), C.c_void_p, C.c_size_t,
                                          C.c_void_p]),
        "gs3_render": (C.c_int, [P(gs3_scene), P(gs3_view), P(gs3_view), P(gs3_consts), C.c_void_p,
                                 P(gs3_mlp), P(gs3_mlp), P(gs3_viewbuf), P(gs3_images), C.c_void_p]),
        "gs3_image_accumulate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_float, C.c_int64, C.c_void_p]),
        "gs3_shadow_splat_views": (C.c_int, [P(gs3_consts), P(gs3_viewbuf), C.c_int32, P(C.c_void_p),
                                             P(C.c_void_p), C.c_void_p]),
        "gs3_render_views": (C.c_int, [P(gs3_scene), P(gs3_view), P(gs3_view), C.c_int32, P(gs3_consts),
                                       P(C.c_void_p), P(gs3_mlp), P(gs3_mlp), P(gs3_viewbuf), P(gs3_images),
                                       C.c_void_p]),
        "gs3_view_poll": (C.c_int, [P(gs3_viewbuf), P(C.c_int32), P(C.c_int64)]),
        "gs3_l1_loss_workspace_size": (C.c_int, [C.c_int64, P(C.c_size_t)]),
        "gs3_l1_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_size_t, C.c_void_p]),
        "gs3_l1_loss_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p, C.c_void_p,
                                          C.c_void_p]),
        "gs3_dssim_loss_workspace_size": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, P(C.c_size_t)]),
        "gs3_dssim_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_float,
                                     C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
        "gs3_adam_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                    C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p]),
        "gs3_grads_clear": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
        "gs3_grads_accumulate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


class Gs3Error(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.gs3_last_error().decode()
        super().__init__(f"{where}: {_lib.gs3_status_string(status).decode()}: {msg}")


def _check(status: int, where: str):
    if status != GS3_OK:
        raise Gs3Error(status, where)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to libgs3 must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to libgs3 must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_consts() -> gs3_consts:
    k = gs3_consts()
    _lib.gs3_consts_default(C.byref(k))
    return k


def make_consts(**kw) -> gs3_consts:
    k = default_consts()
    for name, v in kw.items():
        setattr(k, name, float(v))
    return k


def make_view(view) -> gs3_view:
    """``view`` has eye, target, width, height, fov (radians) and optionally
    projection ("perspective" / "orthographic") and ortho_width."""
    v = gs3_view()
    for i in range(3):
        v.eye[i] = float(view.eye[i])
        v.target[i] = float(view.target[i])
    v.width = int(view.width)
    v.height = int(view.height)
    v.fov = float(view.fov)
    ortho = getattr(view, "projection", "perspective") == "orthographic"
    v.projection = GS3_ORTHOGRAPHIC if ortho else GS3_PERSPECTIVE
    v.ortho_width = float(getattr(view, "ortho_width", 0.0))
    return v


def device_ok() -> bool:
    return bool(_lib.gs3_device_ok())


# ---------------------------------------------------------------- scenes

@dataclasses.dataclass
class DeviceScene:
    """A scene's raw parameters as contiguous float32 device tensors. A
    scene with the paper's shared-basis appearance (``scene.basis``) holds
    rho_s, the basis weights, the latent and the shared basis frames and
    sigmas instead of the per-Gaussian lobes and features."""
    t: Dict[str, torch.Tensor]
    phi: Optional[list]
    psi: Optional[list]
    n: int
    k: int
    appearance: int = GS3_APPEARANCE_LOBES

    @classmethod
    def from_host(cls, scene, device="cuda") -> "DeviceScene":
        names = ["mean", "log_scale", "rot", "opacity_logit", "shade_rot", "albedo"]
        basis = getattr(scene, "basis", None)
        if basis is None:
            names += ["lobe_axis", "lobe_log_sharp", "lobe_amp", "feat"]
        t = {nm: torch.as_tensor(np.ascontiguousarray(getattr(scene, nm), np.float32)).to(device)
             for nm in names}
        if basis is not None:
            src = {"spec_albedo": basis.spec_albedo, "basis_weight": basis.weight, "latent": basis.latent,
                   "basis_rot": basis.basis_rot, "basis_log_sigma": basis.basis_log_sigma}
            for nm in BASIS_NAMES:
                t[nm] = torch.as_tensor(np.ascontiguousarray(src[nm], np.float32)).to(device)

        def mlp(m):
            if m is None:
                return None
            return [(torch.as_tensor(np.ascontiguousarray(w, np.float32)).to(device),
                     torch.as_tensor(np.ascontiguousarray(b, np.float32)).to(device)) for w, b in m.layers]
        k = int(basis.weight.shape[0]) if basis is not None else int(scene.lobe_axis.shape[0])
        return cls(t, mlp(scene.phi), mlp(scene.psi), int(scene.mean.shape[1]), k,
                   GS3_APPEARANCE_BASIS if basis is not None else GS3_APPEARANCE_LOBES)

    @property
    def phi_io(self):
        """(n_in, n_out) of Phi for this scene's appearance model."""
        return (61, 1) if self.appearance == GS3_APPEARANCE_BASIS else (17, 1)

    @property
    def psi_io(self):
        return (60, 3) if self.appearance == GS3_APPEARANCE_BASIS else (22, 3)

    def c_struct(self) -> gs3_scene:
        s = gs3_scene()
        for nm, v in self.t.items():
            setattr(s, nm, _ptr(v))
        s.n = self.n
        s.k = self.k
        s.appearance = self.appearance
        return s

    @staticmethod
    def c_mlp(layers, n_in: int, n_out: int) -> Optional[gs3_mlp]:
        if layers is None:
            return None
        m = gs3_mlp()
        for i, (w, b) in enumerate(layers):
            m.w[i] = _ptr(w).value
            m.b[i] = _ptr(b).value
        m.n_in, m.n_out = n_in, n_out
        return m


class ViewBuffer:
    """Device workspace of one view (projected splats, sort buffers, lists)
    and its host-pinned binning status block (see gs3_viewbuf.status), which
    reports a pair-capacity overflow without a stream synchronisation."""

    def __init__(self, n: int, width: int, height: int, pair_capacity: int, device="cuda",
                 status: bool = True):
        size = C.c_size_t()
        _check(_lib.gs3_view_workspace_size(n, width, height, pair_capacity, C.byref(size)),
               "gs3_view_workspace_size")
        self.storage = torch.empty(size.value + 256, dtype=torch.uint8, device=device)
        base = self.storage.data_ptr()
        off = (-base) % 256
        self.status = torch.zeros(2, dtype=torch.int64, pin_memory=True) if status else None
        self.vb = gs3_viewbuf(C.c_void_p(base + off), size.value, n, width, height, pair_capacity,
                              C.c_void_p(self.status.data_ptr()) if status else None)
        self.n, self.width, self.height, self.capacity = n, width, height, pair_capacity
        self.tiles_x = (width + 15) // 16
        self.tiles_y = (height + 15) // 16


# --------------------------------------------------- C entry points (1:1)

def gs3_project(scene: DeviceScene, view, consts: gs3_consts, depth_mode: int, vb: ViewBuffer):
    v = make_view(view)
    _check(_lib.gs3_project(C.byref(scene.c_struct()), C.byref(v), C.byref(consts), depth_mode,
                            C.byref(vb.vb), _stream()), "gs3_project")


def gs3_bin(ix, iy, rx, ry, depth, vb: ViewBuffer):
    _check(_lib.gs3_bin(_ptr(ix), _ptr(iy), _ptr(rx), _ptr(ry), _ptr(depth), C.byref(vb.vb), _stream()),
           "gs3_bin")


def gs3_preprocess(scene: DeviceScene, view, consts: gs3_consts, depth_mode: int, vb: ViewBuffer):
    v = make_view(view)
    _check(_lib.gs3_preprocess(C.byref(scene.c_struct()), C.byref(v), C.byref(consts), depth_mode,
                               C.byref(vb.vb), _stream()), "gs3_preprocess")


def gs3_preprocess_views(scene: DeviceScene, views: Sequence, depth_modes: Sequence[int], consts: gs3_consts,
                         vbs: Sequence[ViewBuffer]):
    """Projection and binning of several views in one launch sequence."""
    n = len(views)
    if n < 1 or len(depth_modes) != n or len(vbs) != n:
        raise ValueError("one depth mode and one view buffer per view, at least one view")
    va = (gs3_view * n)(*[make_view(v) for v in views])
    ma = (C.c_int32 * n)(*depth_modes)
    ba = (gs3_viewbuf * n)(*[vb.vb for vb in vbs])
    _check(_lib.gs3_preprocess_views(C.byref(scene.c_struct()), va, ma, n, C.byref(consts), ba, _stream()),
           "gs3_preprocess_views")


def gs3_sort(vb: ViewBuffer):
    _check(_lib.gs3_sort(C.byref(vb.vb), _stream()), "gs3_sort")


def gs3_view_pair_count(vb: ViewBuffer) -> int:
    """Pair count of the last binning; raises Gs3Error on overflow (the
    required count is then in ``.required``)."""
    n = C.c_int64()
    st = _lib.gs3_view_pair_count(C.byref(vb.vb), C.byref(n), _stream())
    if st == GS3_PAIR_CAPACITY_EXCEEDED:
        e = Gs3Error(st, "gs3_view_pair_count")
        e.required = int(n.value)
        raise e
    _check(st, "gs3_view_pair_count")
    return int(n.value)


def gs3_view_poll(vb: ViewBuffer):
    """(state, required pairs) of the latest binning from the status block,
    without touching the stream: state is GS3_VIEW_PENDING (not finished on
    the device yet; required = -1), GS3_VIEW_OK or GS3_VIEW_OVERFLOW."""
    st, req = C.c_int32(), C.c_int64()
    _check(_lib.gs3_view_poll(C.byref(vb.vb), C.byref(st), C.byref(req)), "gs3_view_poll")
    return int(st.value), int(req.value)


def gs3_view_lists(vb: ViewBuffer):
    """(tile_start, tile_end, ids, keys) device tensors of the binning."""
    p = gs3_view_pair_count(vb)
    dev = vb.storage.device
    tiles = vb.tiles_x * vb.tiles_y
    ts = torch.empty(tiles, dtype=torch.int32, device=dev)
    te = torch.empty(tiles, dtype=torch.int32, device=dev)
    ids = torch.empty(max(p, 1), dtype=torch.int32, device=dev)
    keys = torch.empty(max(p, 1), dtype=torch.int64, device=dev)
    _check(_lib.gs3_view_lists(C.byref(vb.vb), _ptr(ts), _ptr(te), _ptr(ids), _ptr(keys), _stream()),
           "gs3_view_lists")
    return ts, te, ids[:p], keys[:p]


def gs3_view_splats(vb: ViewBuffer):
    """Projected splats: mean2d [2,n], conic [3,n], opacity [n], depth [n], extent [4,n] int32."""
    dev = vb.storage.device
    n = vb.n
    out = (torch.empty(2, n, device=dev), torch.empty(3, n, device=dev), torch.empty(n, device=dev),
           torch.empty(n, device=dev), torch.empty(4, n, dtype=torch.int32, device=dev))
    _check(_lib.gs3_view_splats(C.byref(vb.vb), *[_ptr(x) for x in out], _stream()), "gs3_view_splats")
    return out


def gs3_view_count_hits(consts: gs3_consts, vb: ViewBuffer, stop_early: bool) -> torch.Tensor:
    """Device int64 tensor [1] with the view's hit count (see gs3.h)."""
    out = torch.empty(1, dtype=torch.int64, device=vb.storage.device)
    _check(_lib.gs3_view_count_hits(C.byref(consts), C.byref(vb.vb), int(bool(stop_early)), _ptr(out), _stream()),
           "gs3_view_count_hits")
    return out


def gs3_shadow_splat(consts: gs3_consts, light_vb: ViewBuffer, num_den: torch.Tensor, T: torch.Tensor):
    _check(_lib.gs3_shadow_splat(C.byref(consts), C.byref(light_vb.vb), _ptr(num_den), _ptr(T), _stream()),
           "gs3_shadow_splat")


def gs3_shadow_den(consts: gs3_consts, light_vb: ViewBuffer, num_den: torch.Tensor):
    _check(_lib.gs3_shadow_den(C.byref(consts), C.byref(light_vb.vb), _ptr(num_den), _stream()), "gs3_shadow_den")


def gs3_shadow_num(consts: gs3_consts, light_vb: ViewBuffer, num_den: torch.Tensor):
    _check(_lib.gs3_shadow_num(C.byref(consts), C.byref(light_vb.vb), _ptr(num_den), _stream()), "gs3_shadow_num")


def gs3_shadow_resolve(light_vb: ViewBuffer, num_den: torch.Tensor, T: torch.Tensor):
    _check(_lib.gs3_shadow_resolve(C.byref(light_vb.vb), _ptr(num_den), _ptr(T), _stream()), "gs3_shadow_resolve")


def gs3_render(scene: DeviceScene, cam, light, consts: gs3_consts, T: torch.Tensor, cam_vb: ViewBuffer,
               images: Dict[str, torch.Tensor], use_mlps: bool = True):
    """``light`` is the light's view: perspective for a point light at its
    eye, orthographic for a directional light."""
    v = make_view(cam)
    lp = make_view(light)
    phi = DeviceScene.c_mlp(scene.phi, *scene.phi_io) if use_mlps else None
    psi = DeviceScene.c_mlp(scene.psi, *scene.psi_io) if use_mlps else None
    im = gs3_images(*[_ptr(images[k]) for k in ("final", "S", "Sh", "R", "T_final", "n_contrib", "colour")])
    _check(_lib.gs3_render(C.byref(scene.c_struct()), C.byref(v), C.byref(lp), C.byref(consts), _ptr(T),
                           C.byref(phi) if phi is not None else None,
                           C.byref(psi) if psi is not None else None,
                           C.byref(cam_vb.vb), C.byref(im), _stream()), "gs3_render")


def gs3_shade(scene: DeviceScene, cam, light, cam_vb: ViewBuffer, colour: torch.Tensor, use_mlps: bool = True):
    v = make_view(cam)
    lp = make_view(light)
    psi = DeviceScene.c_mlp(scene.psi, *scene.psi_io) if use_mlps else None
    _check(_lib.gs3_shade(C.byref(scene.c_struct()), C.byref(v), C.byref(lp),
                          C.byref(psi) if psi is not None else None, C.byref(cam_vb.vb), _ptr(colour), _stream()),
           "gs3_shade")


def gs3_render_shaded(scene: DeviceScene, cam, light, consts: gs3_consts, T: torch.Tensor, cam_vb: ViewBuffer,
                      images: Dict[str, torch.Tensor], use_mlps: bool = True):
    v = make_view(cam)
    lp = make_view(light)
    phi = DeviceScene.c_mlp(scene.phi, *scene.phi_io) if use_mlps else None
    im = gs3_images(*[_ptr(images[k]) for k in ("final", "S", "Sh", "R", "T_final", "n_contrib", "colour")])
    _check(_lib.gs3_render_shaded(C.byref(scene.c_struct()), C.byref(v), C.byref(lp), C.byref(consts), _ptr(T),
                                  C.byref(phi) if phi is not None else None, C.byref(cam_vb.vb), C.byref(im),
                                  _stream()), "gs3_render_shaded")


def gs3_shadow_splat_views(consts: gs3_consts, light_vbs: Sequence[ViewBuffer], num_dens: Sequence[torch.Tensor],
                           Ts: Sequence[torch.Tensor]):
    """Shadow splats of several light views in one launch sequence."""
    n = len(light_vbs)
    if n < 1 or len(num_dens) != n or len(Ts) != n:
        raise ValueError("one num_den and one T per light view, at least one view")
    ba = (gs3_viewbuf * n)(*[vb.vb for vb in light_vbs])
    nd = (C.c_void_p * n)(*[_ptr(t).value for t in num_dens])
    ta = (C.c_void_p * n)(*[_ptr(t).value for t in Ts])
    _check(_lib.gs3_shadow_splat_views(C.byref(consts), ba, n, nd, ta, _stream()), "gs3_shadow_splat_views")


def gs3_render_views(scene: DeviceScene, cams: Sequence, lights: Sequence, consts: gs3_consts,
                     Ts: Sequence[torch.Tensor], cam_vbs: Sequence[ViewBuffer],
                     images: Sequence[Dict[str, torch.Tensor]], use_mlps: bool = True):
    """Shading, MLPs and camera splats of several (camera, light) views in
    one launch sequence."""
    n = len(cams)
    if n < 1 or len(lights) != n or len(Ts) != n or len(cam_vbs) != n or len(images) != n:
        raise ValueError("one light, T, camera buffer and image set per camera, at least one camera")
    ca = (gs3_view * n)(*[make_view(v) for v in cams])
    la = (gs3_view * n)(*[make_view(v) for v in lights])
    ta = (C.c_void_p * n)(*[_ptr(t).value for t in Ts])
    ba = (gs3_viewbuf * n)(*[vb.vb for vb in cam_vbs])
    ia = (gs3_images * n)(*[gs3_images(*[_ptr(im[k]) for k in ("final", "S", "Sh", "R", "T_final", "n_contrib",
                                                                 "colour")]) for im in images])
    phi = DeviceScene.c_mlp(scene.phi, *scene.phi_io) if use_mlps else None
    psi = DeviceScene.c_mlp(scene.psi, *scene.psi_io) if use_mlps else None
    _check(_lib.gs3_render_views(C.byref(scene.c_struct()), ca, la, n, C.byref(consts), ta,
                                 C.byref(phi) if phi is not None else None,
                                 C.byref(psi) if psi is not None else None, ba, ia, _stream()),
           "gs3_render_views")


def l1_workspace(count: int, device="cuda") -> torch.Tensor:
    size = C.c_size_t()
    _check(_lib.gs3_l1_loss_workspace_size(int(count), C.byref(size)), "gs3_l1_loss_workspace_size")
    return torch.empty(size.value + 256, dtype=torch.uint8, device=device)


def gs3_l1_loss(pred: torch.Tensor, target: torch.Tensor, scale: float, loss: torch.Tensor,
                grad: Optional[torch.Tensor], ws: torch.Tensor):
    """loss[0] = scale * sum |pred - target|; grad = scale * sign(pred - target)
    (if given). All float32 device tensors with pred's element count."""
    count = pred.numel()
    if target.numel() != count or (grad is not None and grad.numel() != count):
        raise ValueError("pred, target and grad must have the same number of elements")
    for t in (pred, target, loss) + ((grad,) if grad is not None else ()):
        if t.dtype != torch.float32:
            raise ValueError("gs3_l1_loss takes float32 tensors")
    wsp, wsb = _aligned(ws)
    _check(_lib.gs3_l1_loss(_ptr(pred), _ptr(target), count, float(scale), _ptr(loss), _ptr(grad), wsp, wsb,
                            _stream()), "gs3_l1_loss")


def gs3_l1_loss_noalloc(pred: torch.Tensor, target: torch.Tensor, scale: float, loss: torch.Tensor,
                        grad: Optional[torch.Tensor]):
    """gs3_l1_loss without a workspace (the library's own per-device
    scratch; at most 33,554,432 elements; calls on one device must not
    overlap)."""
    count = pred.numel()
    if target.numel() != count or (grad is not None and grad.numel() != count):
        raise ValueError("pred, target and grad must have the same number of elements")
    _check(_lib.gs3_l1_loss_noalloc(_ptr(pred), _ptr(target), count, float(scale), _ptr(loss), _ptr(grad),
                                    _stream()), "gs3_l1_loss_noalloc")


def dssim_workspace(channels: int, height: int, width: int, device="cuda") -> torch.Tensor:
    size = C.c_size_t()
    _check(_lib.gs3_dssim_loss_workspace_size(channels, height, width, C.byref(size)),
           "gs3_dssim_loss_workspace_size")
    return torch.empty(size.value + 256, dtype=torch.uint8, device=device)


def gs3_dssim_loss(pred: torch.Tensor, target: torch.Tensor, scale: float, loss: torch.Tensor,
                   grad: Optional[torch.Tensor], ws: torch.Tensor, accumulate: bool = False):
    """loss[0] = scale * sum (1 - SSIM) over the [C, H, W] images; grad (if
    given) gets (or, with accumulate, adds) its gradient."""
    if pred.dim() != 3 or pred.shape != target.shape or (grad is not None and grad.shape != pred.shape):
        raise ValueError("pred, target and grad must be [C, H, W] of one shape")
    c, h, w = pred.shape
    wsp, wsb = _aligned(ws)
    _check(_lib.gs3_dssim_loss(_ptr(pred), _ptr(target), c, h, w, float(scale), _ptr(loss), _ptr(grad),
                               int(bool(accumulate)), wsp, wsb, _stream()), "gs3_dssim_loss")


def gs3_adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
                  lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15):
    n = param.numel()
    if not (grad.numel() == m.numel() == v.numel() == n):
        raise ValueError("param, grad, m and v must have one size")
    _check(_lib.gs3_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), n, int(step), float(lr), float(beta1),
                              float(beta2), float(eps), _stream()), "gs3_adam_step")


def gs3_image_accumulate(dst: torch.Tensor, src: torch.Tensor, weight: float):
    """dst += weight * src (float32 device tensors of one size)."""
    if dst.dtype != torch.float32 or src.dtype != torch.float32 or dst.numel() != src.numel():
        raise ValueError("images must be float32 of one size")
    _check(_lib.gs3_image_accumulate(_ptr(dst), _ptr(src), float(weight), dst.numel(), _stream()),
           "gs3_image_accumulate")


def gs3_grads_clear(g: torch.Tensor):
    if g.dtype != torch.float32:
        raise ValueError("gradients are float32")
    _check(_lib.gs3_grads_clear(_ptr(g), g.numel(), _stream()), "gs3_grads_clear")


def gs3_grads_accumulate(dst: torch.Tensor, src: torch.Tensor):
    if dst.dtype != torch.float32 or src.dtype != torch.float32 or dst.numel() != src.numel():
        raise ValueError("gradient sets must be float32 of one size")
    _check(_lib.gs3_grads_accumulate(_ptr(dst), _ptr(src), dst.numel(), _stream()), "gs3_grads_accumulate")


class DeviceGrads:
    """Gradient tensors shaped like a DeviceScene's (zeroed), for
    gs3_render_backward. They are views of one flat buffer (each slice
    256-byte aligned), so clearing or summing a whole set is one kernel."""

    def __init__(self, scene: DeviceScene, use_mlps: bool = True):
        like = list(scene.t.values())
        mlps = [m if (m is not None and use_mlps) else None for m in (scene.phi, scene.psi)]
        for m in mlps:
            if m is not None:
                for w, b in m:
                    like += [w, b]
        offs, total = [], 0
        for v in like:
            offs.append(total)
            total += (v.numel() + 63) // 64 * 64
        self.flat = torch.empty(max(total, 1), dtype=torch.float32, device=like[0].device)
        gs3_grads_clear(self.flat)
        views = iter(self.flat[o:o + v.numel()].view(v.shape) for o, v in zip(offs, like))
        self.t = {nm: next(views) for nm in scene.t}
        self.phi, self.psi = [None if m is None else [(next(views), next(views)) for _ in m] for m in mlps]

    def zero_(self) -> "DeviceGrads":
        gs3_grads_clear(self.flat)
        return self

    def add_(self, other: "DeviceGrads") -> "DeviceGrads":
        """Adds another set of the same scene and MLP configuration."""
        gs3_grads_accumulate(self.flat, other.flat)
        return self

    def c_struct(self) -> gs3_grads:
        g = gs3_grads()
        for nm, v in self.t.items():
            setattr(g, nm, _ptr(v).value)
        for mlp, wn, bn in ((self.phi, "phi_w", "phi_b"), (self.psi, "psi_w", "psi_b")):
            if mlp is not None:
                for i, (w, b) in enumerate(mlp):
                    getattr(g, wn)[i] = _ptr(w).value
                    getattr(g, bn)[i] = _ptr(b).value
        return g


def backward_workspace(n: int, light_width: int, light_height: int, device="cuda",
                       appearance: int = GS3_APPEARANCE_LOBES) -> torch.Tensor:
    size = C.c_size_t()
    _check(_lib.gs3_backward_workspace_size_for(appearance, n, light_width, light_height, C.byref(size)),
           "gs3_backward_workspace_size_for")
    return torch.empty(size.value + 256, dtype=torch.uint8, device=device)


def _aligned(buf: torch.Tensor):
    base = buf.data_ptr()
    off = (-base) % 256
    return C.c_void_p(base + off), buf.numel() - off


def gs3_render_backward(scene: DeviceScene, cam, light, consts: gs3_consts, T: torch.Tensor,
                        num_den: torch.Tensor, light_vb: ViewBuffer, cam_vb: ViewBuffer,
                        images: Dict[str, torch.Tensor], dL_dfinal: torch.Tensor, grads: DeviceGrads,
                        ws: torch.Tensor, use_mlps: bool = True):
    cv, lv = make_view(cam), make_view(light)
    phi = DeviceScene.c_mlp(scene.phi, *scene.phi_io) if use_mlps else None
    psi = DeviceScene.c_mlp(scene.psi, *scene.psi_io) if use_mlps else None
    im = gs3_images(*[_ptr(images[k]) for k in ("final", "S", "Sh", "R", "T_final", "n_contrib", "colour")])
    g = grads.c_struct()
    wsp, wsb = _aligned(ws)
    _check(_lib.gs3_render_backward(C.byref(scene.c_struct()), C.byref(cv), C.byref(lv), C.byref(consts), _ptr(T),
                                    _ptr(num_den), C.byref(phi) if phi is not None else None,
                                    C.byref(psi) if psi is not None else None, C.byref(light_vb.vb),
                                    C.byref(cam_vb.vb), C.byref(im), _ptr(dL_dfinal), C.byref(g), wsp, wsb,
                                    _stream()), "gs3_render_backward")


# ------------------------------------------------------------- renderer

class Renderer:
    """One relit frame (Sec. 4): light preprocess, shadow splat, camera
    preprocess, shading + MLPs + camera splat. Buffers are allocated on
    first use and grown when a binning needs more pairs."""

    def __init__(self, scene: DeviceScene, consts: Optional[gs3_consts] = None, use_mlps: bool = True,
                 pair_capacity: Optional[int] = None, batch_views: bool = False):
        self.scene = scene
        self.batch_views = batch_views
        self.consts = consts if consts is not None else default_consts()
        self.use_mlps = use_mlps and scene.phi is not None
        self.capacity_hint = pair_capacity
        self.vbs: Dict[tuple, ViewBuffer] = {}
        self.dev = scene.t["mean"].device
        n = scene.n
        self.num_den = torch.empty(2, max(n, 1), device=self.dev)
        self.T = torch.empty(max(n, 1), device=self.dev)
        self.images: Dict[tuple, Dict[str, torch.Tensor]] = {}
        self.bwd_ws: Optional[torch.Tensor] = None
        self.side = None

    def _vb(self, role: str, w: int, h: int, capacity: int) -> ViewBuffer:
        key = (role, w, h)
        vb = self.vbs.get(key)
        if vb is None or vb.capacity < capacity:
            vb = ViewBuffer(self.scene.n, w, h, capacity, self.dev)
            self.vbs[key] = vb
        return vb

    def _preprocess(self, role: str, view, mode: int, check: bool) -> ViewBuffer:
        key = (role, view.width, view.height)
        vb = self.vbs.get(key)
        if vb is None:
            cap = self.capacity_hint or max(1 << 16, 32 * self.scene.n)
            vb = self._vb(role, view.width, view.height, cap)
        gs3_preprocess(self.scene, view, self.consts, mode, vb)
        if check:
            try:
                gs3_view_pair_count(vb)
            except Gs3Error as e:
                if e.status != GS3_PAIR_CAPACITY_EXCEEDED:
                    raise
                vb = self._vb(role, view.width, view.height, int(e.required * 1.25) + 4096)
                gs3_preprocess(self.scene, view, self.consts, mode, vb)
                gs3_view_pair_count(vb)
        return vb

    def _preprocess_pair(self, light, cam, check: bool):
        """Light (distance keys) and camera (z keys) preprocess in one
        launch sequence (gs3_preprocess_views); with ``check``, a view whose
        binning overflowed is grown and preprocessed again on its own."""
        vbs = []
        for role, view in (("light", light), ("cam", cam)):
            vb = self.vbs.get((role, view.width, view.height))
            if vb is None:
                cap = self.capacity_hint or max(1 << 16, 32 * self.scene.n)
                vb = self._vb(role, view.width, view.height, cap)
            vbs.append(vb)
        gs3_preprocess_views(self.scene, [light, cam], [GS3_DEPTH_DIST, GS3_DEPTH_Z], self.consts, vbs)
        if check:
            for i, (role, view, mode) in enumerate((("light", light, GS3_DEPTH_DIST), ("cam", cam, GS3_DEPTH_Z))):
                try:
                    gs3_view_pair_count(vbs[i])
                except Gs3Error as e:
                    if e.status != GS3_PAIR_CAPACITY_EXCEEDED:
                        raise
                    vbs[i] = self._vb(role, view.width, view.height, int(e.required * 1.25) + 4096)
                    gs3_preprocess(self.scene, view, self.consts, mode, vbs[i])
                    gs3_view_pair_count(vbs[i])
        return vbs[0], vbs[1]

    def _images(self, w: int, h: int):
        key = (w, h)
        im = self.images.get(key)
        if im is None:
            d = self.dev
            im = {"final": torch.empty(3, h, w, device=d), "S": torch.empty(3, h, w, device=d),
                  "Sh": torch.empty(h, w, device=d), "R": torch.empty(3, h, w, device=d),
                  "T_final": torch.empty(h, w, device=d),
                  "n_contrib": torch.empty(h, w, dtype=torch.int32, device=d),
                  "colour": torch.empty(8, max(self.scene.n, 1), device=d)}
            self.images[key] = im
        return im

    def render_shadowed(self, cam, light, T: torch.Tensor, check: bool = True) -> Dict[str, torch.Tensor]:
        """Relit frame for camera ``cam`` under the point light of view
        ``light`` whose shadow values ``T`` [n] were already computed (by a
        render of the same light view): only the camera path runs (camera
        preprocess, shading + MLPs, camera splat). Used to share one shadow
        splat among requests with the same light."""
        cvb = self._preprocess("cam", cam, GS3_DEPTH_Z, check)
        im = self._images(cam.width, cam.height)
        gs3_render(self.scene, cam, light, self.consts, T, cvb, im, self.use_mlps)
        out = dict(im)
        out["T"] = T
        return out

    def render(self, cam, light, check: bool = True, overlap: bool = True,
               events: Optional[Dict[str, torch.cuda.Event]] = None,
               batch: Optional[bool] = None) -> Dict[str, torch.Tensor]:
        """Relit frame for camera view ``cam`` and the point light of view
        ``light`` (its eye is the light position). ``check`` verifies (with a
        host sync) that no binning overflowed its pair capacity.

        With ``overlap`` the independent parts of the frame run on two side
        streams (default priority) joined by events: the camera preprocess
        from the start of the frame, the shadow denominator once the light
        lists exist, while the caller's stream runs the light preprocess and
        the shadow numerator, then the resolve and the camera pass; the
        shading and Psi (independent of the shadow values) run on the camera
        side stream, only Phi waits for the resolve. The light path is
        issued first: one frame at a time the host's launches would
        otherwise delay it. The numerator's tail occupies few CUs, which
        the other two fill. Results
        are the same as with ``overlap=False`` (one stream, in order).
        ``events`` (optional) gets "num0"/"num1" recorded around the shadow
        numerator on the caller's stream, and "den0"/"den1" (when present)
        around the denominator on the stream it runs on. With ``batch``
        (default: the renderer's ``batch_views``) the two views are
        preprocessed in one launch sequence (gs3_preprocess_views); with
        ``overlap`` as well the denominator and the shading then run on the
        side streams after it."""
        main = torch.cuda.current_stream()
        batch = self.batch_views if batch is None else batch
        if batch and (not overlap or check):
            lvb, cvb = self._preprocess_pair(light, cam, check)
            if events is not None and "den0" in events:
                events["den0"].record(main)
            gs3_shadow_den(self.consts, lvb, self.num_den)
            if events is not None and "den1" in events:
                events["den1"].record(main)
            if events is not None:
                events["num0"].record(main)
            gs3_shadow_num(self.consts, lvb, self.num_den)
            if events is not None:
                events["num1"].record(main)
            gs3_shadow_resolve(lvb, self.num_den, self.T)
        elif not overlap or check:
            lvb = self._preprocess("light", light, GS3_DEPTH_DIST, check)
            if events is not None and "den0" in events:
                events["den0"].record(main)
            gs3_shadow_den(self.consts, lvb, self.num_den)
            if events is not None and "den1" in events:
                events["den1"].record(main)
            if events is not None:
                events["num0"].record(main)
            gs3_shadow_num(self.consts, lvb, self.num_den)
            if events is not None:
                events["num1"].record(main)
            gs3_shadow_resolve(lvb, self.num_den, self.T)
            cvb = self._preprocess("cam", cam, GS3_DEPTH_Z, check)
        else:
            if self.side is None:
                self.side = (torch.cuda.Stream(), torch.cuda.Stream())
                self.side_events = (torch.cuda.Event(), torch.cuda.Event())
            s_den, s_cam = self.side
            ev_start, ev_light = self.side_events
            im = self._images(cam.width, cam.height)
            # the light path (preprocess, numerator, resolve) is the frame's
            # critical path, so it is issued first; the side streams start
            # after everything already on the caller's stream (the previous
            # frame still reads these buffers), not after this frame's work
            ev_start.record(main)
            if batch:
                lvb, cvb = self._preprocess_pair(light, cam, False)
            else:
                lvb = self._preprocess("light", light, GS3_DEPTH_DIST, False)
            ev_light.record(main)
            s_den.wait_event(ev_light)
            with torch.cuda.stream(s_den):
                if events is not None and "den0" in events:
                    events["den0"].record(s_den)
                gs3_shadow_den(self.consts, lvb, self.num_den)
                if events is not None and "den1" in events:
                    events["den1"].record(s_den)
            if events is not None:
                events["num0"].record(main)
            gs3_shadow_num(self.consts, lvb, self.num_den)
            if events is not None:
                events["num1"].record(main)
            s_cam.wait_event(ev_light if batch else ev_start)
            with torch.cuda.stream(s_cam):
                if not batch:
                    cvb = self._preprocess("cam", cam, GS3_DEPTH_Z, False)
                gs3_shade(self.scene, cam, light, cvb, im["colour"], self.use_mlps)
            main.wait_stream(s_den)
            gs3_shadow_resolve(lvb, self.num_den, self.T)
            main.wait_stream(s_cam)
            gs3_render_shaded(self.scene, cam, light, self.consts, self.T, cvb, im, self.use_mlps)
            out = dict(im)
            out["T"] = self.T
            out["num_den"] = self.num_den
            return out
        im = self._images(cam.width, cam.height)
        gs3_render(self.scene, cam, light, self.consts, self.T, cvb, im, self.use_mlps)
        out = dict(im)
        out["T"] = self.T
        out["num_den"] = self.num_den
        return out

    def render_env(self, cam, lights: Sequence, weights: Sequence[float], check: bool = True) -> torch.Tensor:
        """Environment lighting (Sec. 4.5): the weighted sum of the relit
        frames of ``cam`` under each light of ``lights`` (directional lights:
        orthographic light views, synth.environment_lights) with
        ``weights``. The camera preprocess runs once; each light runs its
        own light preprocess, shadow splat, shading and camera splat, and
        its frame is added into the result with gs3_image_accumulate.
        Returns a new [3, H, W] tensor."""
        if len(lights) != len(weights) or not len(lights):
            raise ValueError("one weight per light, at least one light")
        cvb = self._preprocess("cam", cam, GS3_DEPTH_Z, check)
        im = self._images(cam.width, cam.height)
        env = torch.empty(3, cam.height, cam.width, device=self.dev)
        gs3_grads_clear(env)
        for light, w in zip(lights, weights):
            lvb = self._preprocess("light", light, GS3_DEPTH_DIST, check)
            gs3_shadow_den(self.consts, lvb, self.num_den)
            gs3_shadow_num(self.consts, lvb, self.num_den)
            gs3_shadow_resolve(lvb, self.num_den, self.T)
            gs3_render(self.scene, cam, light, self.consts, self.T, cvb, im, self.use_mlps)
            gs3_image_accumulate(env, im["final"], float(w))
        return env

    def backward(self, cam, light, dL_dfinal: torch.Tensor, grads: Optional["DeviceGrads"] = None) -> "DeviceGrads":
        """Adjoint of the last ``render(cam, light)`` of this renderer (its
        buffers must not have been reused since): adds dL/d(parameters) for
        the given dL/dfinal [3, H, W] into ``grads`` (new zeros if None)."""
        if tuple(dL_dfinal.shape) != (3, cam.height, cam.width) or dL_dfinal.dtype != torch.float32:
            raise ValueError(f"dL_dfinal must be float32 [3, {cam.height}, {cam.width}], got "
                             f"{dL_dfinal.dtype} {tuple(dL_dfinal.shape)}")
        if grads is None:
            grads = DeviceGrads(self.scene, self.use_mlps)
        app = self.scene.appearance
        if self.bwd_ws is None:
            self.bwd_ws = backward_workspace(self.scene.n, light.width, light.height, self.dev, app)
        need = C.c_size_t()
        _check(_lib.gs3_backward_workspace_size_for(app, self.scene.n, light.width, light.height, C.byref(need)),
               "gs3_backward_workspace_size_for")
        if self.bwd_ws.numel() < need.value + 256:
            self.bwd_ws = backward_workspace(self.scene.n, light.width, light.height, self.dev, app)
        lvb = self.vbs[("light", light.width, light.height)]
        cvb = self.vbs[("cam", cam.width, cam.height)]
        gs3_render_backward(self.scene, cam, light, self.consts, self.T, self.num_den, lvb, cvb,
                            self._images(cam.width, cam.height), dL_dfinal.contiguous(), grads, self.bwd_ws,
                            self.use_mlps)
        return grads

    def overflowed(self) -> bool:
        """True if any view's last binning exceeded its capacity. Read from
        the views' status blocks without a synchronisation once their
        binnings have finished; a binning still pending on the device is
        waited for (gs3_view_pair_count)."""
        for vb in self.vbs.values():
            if vb.status is not None:
                state, _ = gs3_view_poll(vb)
                if state == GS3_VIEW_OVERFLOW:
                    return True
                if state == GS3_VIEW_OK:
                    continue
            try:
                gs3_view_pair_count(vb)
            except Gs3Error as e:
                if e.status == GS3_PAIR_CAPACITY_EXCEEDED:
                    return True
                raise
        return False


# ------------------------------------------------------------ autograd

SCENE_FIELDS = ("mean", "log_scale", "rot", "opacity_logit", "shade_rot", "albedo", "lobe_axis",
                "lobe_log_sharp", "lobe_amp", "feat")


def scene_parameters(scene: DeviceScene) -> list:
    """The tensors a RelitRender call differentiates: the scene's raw
    parameters, then Phi's and Psi's (W, b) per layer."""
    ps = list(scene.t.values())
    for m in (scene.phi, scene.psi):
        if m is not None:
            for w, b in m:
                ps += [w, b]
    return ps


class RelitRender(torch.autograd.Function):
    """final = render(scene, cam, light) with the hand-written adjoint
    (gs3_render_backward) as its backward. ``renderer`` holds the forward
    state until the backward runs, so use one Renderer per pending call
    (e.g. one per element of a batch)."""

    @staticmethod
    def forward(ctx, renderer: "Renderer", cam, light, *params):
        out = renderer.render(cam, light, check=True)
        ctx.renderer, ctx.cam, ctx.light = renderer, cam, light
        return out["final"].clone()

    @staticmethod
    def backward(ctx, dfinal):
        r = ctx.renderer
        g = r.backward(ctx.cam, ctx.light, dfinal)
        outs = [g.t[nm] for nm in r.scene.t]
        for gm, sm in ((g.phi, r.scene.phi), (g.psi, r.scene.psi)):
            if sm is None:
                continue
            if gm is None:
                outs += [None] * (2 * len(sm))
            else:
                for w, b in gm:
                    outs += [w, b]
        return (None, None, None, *outs)


def relit_render(renderer: "Renderer", cam, light) -> torch.Tensor:
    """Differentiable relit frame [3, H, W] (see RelitRender)."""
    return RelitRender.apply(renderer, cam, light, *scene_parameters(renderer.scene))


def render_batched(renderers: Sequence["Renderer"], cams: Sequence, lights: Sequence,
                   shadows: Optional[Sequence[Optional[torch.Tensor]]] = None) -> list:
    """Relit frames of several (camera, light) requests with one launch
    sequence per stage: the light and camera views of every request are
    projected and binned together (gs3_preprocess_views), the light views'
    shadow splats run together (gs3_shadow_splat_views) and so do the
    shading, MLPs and camera splats (gs3_render_views). Request i uses the
    buffers of ``renderers[i]`` (all of one scene). Requests whose light view
    is the same share one shadow pass; with ``shadows[i]`` given, request i
    uses those shadow values and runs no light pass. Returns each request's
    output dict (its renderer's images and T). No host synchronisation."""
    n = len(cams)
    if n < 1 or len(renderers) != n or len(lights) != n:
        raise ValueError("one renderer and one light per camera, at least one request")
    shadows = list(shadows) if shadows is not None else [None] * n
    r0 = renderers[0]
    scene, consts = r0.scene, r0.consts

    def vb(r, role, view):
        got = r.vbs.get((role, view.width, view.height))
        if got is None:
            got = r._vb(role, view.width, view.height, r.capacity_hint or max(1 << 16, 32 * scene.n))
        return got

    def key(light):
        return (tuple(float(x) for x in light.eye), tuple(float(x) for x in light.target), light.width,
                light.height, float(light.fov), light.projection, float(light.ortho_width))
    owner: Dict[tuple, int] = {}     # light view -> request running its shadow pass
    for i in range(n):
        if shadows[i] is None:
            owner.setdefault(key(lights[i]), i)
    passes = sorted(owner.values())
    views, modes, vbs = [], [], []
    for i in passes:
        views.append(lights[i]); modes.append(GS3_DEPTH_DIST); vbs.append(vb(renderers[i], "light", lights[i]))
    cvbs = [vb(renderers[i], "cam", cams[i]) for i in range(n)]
    views += list(cams); modes += [GS3_DEPTH_Z] * n; vbs += cvbs
    gs3_preprocess_views(scene, views, modes, consts, vbs)
    if passes:
        gs3_shadow_splat_views(consts, vbs[:len(passes)], [renderers[i].num_den for i in passes],
                               [renderers[i].T for i in passes])
    Ts = [shadows[i] if shadows[i] is not None else renderers[owner[key(lights[i])]].T for i in range(n)]
    ims = [renderers[i]._images(cams[i].width, cams[i].height) for i in range(n)]
    gs3_render_views(scene, cams, lights, consts, Ts, cvbs, ims, r0.use_mlps)
    outs = []
    for i in range(n):
        o = dict(ims[i])
        o["T"] = Ts[i]
        outs.append(o)
    return outs


class EnvPipeline:
    """Environment frames (Sec. 4.5) with several lights in flight: light l
    runs on slot l % slots, each slot a Renderer (its own light and camera
    buffers) on its own stream, so one light's shadow numerator tails off
    while the next lights' passes fill the device. Each slot runs
    Renderer.render_env over its lights (one camera preprocess per slot);
    the slots' weighted sums are added in slot order on the caller's stream,
    so the result does not depend on timing."""

    def __init__(self, scene: DeviceScene, slots: int = 4, consts: Optional[gs3_consts] = None,
                 use_mlps: bool = True, pair_capacity: Optional[int] = None):
        if slots < 1:
            raise ValueError("at least one slot")
        self.renderers = [Renderer(scene, consts, use_mlps, pair_capacity) for _ in range(slots)]
        self.streams = [torch.cuda.Stream() for _ in range(slots)]

    def render(self, cam, lights: Sequence, weights: Sequence[float], check: bool = True) -> torch.Tensor:
        """The weighted sum of the relit frames of ``cam`` under ``lights``
        (as Renderer.render_env). Returns a new [3, H, W] tensor on the
        caller's stream."""
        if len(lights) != len(weights) or not len(lights):
            raise ValueError("one weight per light, at least one light")
        cur = torch.cuda.current_stream()
        start = torch.cuda.Event()
        start.record(cur)
        S = len(self.renderers)
        parts = []
        for k in range(min(S, len(lights))):
            st = self.streams[k]
            st.wait_event(start)
            with torch.cuda.stream(st):
                part = self.renderers[k].render_env(cam, lights[k::S], weights[k::S], check)
            parts.append((part, st))
        for part, st in parts:
            cur.wait_stream(st)
            part.record_stream(cur)
        env = parts[0][0]
        for part, _ in parts[1:]:
            gs3_image_accumulate(env, part, 1.0)
        return env


class FramePipeline:
    """A stream of relit frames with `depth` frames in flight: frame i runs
    on renderer i % depth (its own buffers) and its own stream, so the next
    frame's light pass fills the device while the previous frame's shadow
    numerator tails off and its camera pass runs. Each frame is the same
    computation as Renderer.render; a renderer's buffers are reused `depth`
    frames later, after its previous frame on the same stream."""

    def __init__(self, scene: DeviceScene, depth: int = 2, consts: Optional[gs3_consts] = None,
                 use_mlps: bool = True, pair_capacity: Optional[int] = None, batch_views: bool = False):
        self.renderers = [Renderer(scene, consts, use_mlps, pair_capacity, batch_views) for _ in range(depth)]
        self.streams = [torch.cuda.Stream() for _ in range(depth)]
        self.i = 0

    def warm(self, cam, light):
        """Size every renderer's buffers for this view pair (host syncs)."""
        for r, s in zip(self.renderers, self.streams):
            with torch.cuda.stream(s):
                r.render(cam, light, check=True)
        torch.cuda.synchronize()

    def render(self, cam, light, events: Optional[Dict[str, torch.cuda.Event]] = None,
               overlap: bool = True) -> Dict[str, torch.Tensor]:
        k = self.i % len(self.renderers)
        self.i += 1
        with torch.cuda.stream(self.streams[k]):
            return self.renderers[k].render(cam, light, check=False, overlap=overlap, events=events)

    def render_group(self, cams: Sequence, lights: Sequence) -> list:
        """Several frames as one batch (``render_batched``): one launch
        sequence per stage for all of them, on the stream of the group's
        first renderer. Groups take consecutive renderers, so a renderer's
        buffers are reused only after `depth` frames, on the same stream."""
        g = len(cams)
        k0 = self.i % len(self.renderers)
        if k0 + g > len(self.renderers):
            k0 = 0
            self.i = 0
        self.i += g
        rnds = self.renderers[k0:k0 + g]
        with torch.cuda.stream(self.streams[k0]):
            return render_batched(rnds, cams, lights)

    def overflowed(self) -> bool:
        return any(r.overflowed() for r in self.renderers)
