"""Optimisation step of the relightable representation (Sec. 4.4).

One step renders a batch of (camera, light) views, takes the loss
L = (1 - lambda) L1 + lambda D-SSIM (Eq. 9, lambda = 0.2) of each against
its target image, runs the hand-written adjoint of every view, and applies
one Adam update (momentum 0.9) per parameter tensor. The first stage of the
paper's schedule limits the appearance to the Lambertian term: the
library then evaluates no angular lobes (scene k = 0), and the lobes get no
gradient and no update. Every step of this runs in the library's kernels
(gs3_l1_loss, gs3_dssim_loss, gs3_render_backward, gs3_grads_clear,
gs3_grads_accumulate, gs3_adam_step); torch holds the buffers and streams.

Learning rates: 0.01 for the albedo and the lobe amplitudes (rho_d,
rho_s), 0.01 for the lobe axes and sharpness, decayed exponentially from
0.01 at 40K iterations to 1e-4 at 90K and held there (the paper's figures);
the geometry and the MLPs take the rates of the Gaussian-splatting recipe
the paper follows (positions 1.6e-4, log-scales 5e-3, rotations 1e-3,
opacity logits 5e-2), features and MLP weights 1e-3, shading rotations 1e-3.
A scene with the paper's shared-basis appearance trains rho_s and the basis
weights at 0.01, the latent at 1e-3, and the basis frames and sigmas on the
angular-Gaussian schedule; in the first stage (k = 0) the specular
parameters get no gradient and no update.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import gs3

LOSS_LAMBDA = 0.2
STAGE1_ITERS = 15_000          # Lambertian-only iterations (Sec. 4.4)

BASE_LR = {"mean": 1.6e-4, "log_scale": 5e-3, "rot": 1e-3, "opacity_logit": 5e-2, "shade_rot": 1e-3,
           "albedo": 1e-2, "lobe_axis": 1e-2, "lobe_log_sharp": 1e-2, "lobe_amp": 1e-2, "feat": 1e-3,
           "mlp": 1e-3, "spec_albedo": 1e-2, "basis_weight": 1e-2, "latent": 1e-3, "basis_rot": 1e-2,
           "basis_log_sigma": 1e-2}
# angular-Gaussian shape parameters (the decayed schedule) and the specular
# parameters frozen in the Lambertian stage
LOBE_SHAPE = ("lobe_axis", "lobe_log_sharp", "basis_rot", "basis_log_sigma")
LOBES = ("lobe_axis", "lobe_log_sharp", "lobe_amp", "spec_albedo", "basis_weight", "basis_rot", "basis_log_sigma")


def lobe_lr(it: int) -> float:
    """0.01 up to 40K iterations, exponential decay to 1e-4 at 90K, then 1e-4."""
    if it < 40_000:
        return 1e-2
    if it >= 90_000:
        return 1e-4
    f = (it - 40_000) / 50_000.0
    return math.exp((1 - f) * math.log(1e-2) + f * math.log(1e-4))


class Trainer:
    """Adam over every tensor of a DeviceScene (raw parameters and both
    MLPs), views of a batch spread over `lanes` concurrent renderers."""

    def __init__(self, scene: gs3.DeviceScene, lanes: int = 4, lam: float = LOSS_LAMBDA,
                 stage1_iters: int = STAGE1_ITERS, lr: Optional[Dict[str, float]] = None):
        self.scene = scene
        self.k_full = scene.k
        self.lam = lam
        self.stage1_iters = stage1_iters
        self.lr = dict(BASE_LR, **(lr or {}))
        self.lanes = lanes
        self.rnds = [gs3.Renderer(scene) for _ in range(lanes)]
        self.grads = [gs3.DeviceGrads(scene) for _ in range(lanes)]
        self.streams = [torch.cuda.Stream() for _ in range(lanes)]
        self.it = 0
        self.params = self._tensors(scene.t, scene.phi, scene.psi)
        g0 = self.grads[0]
        self.gtens = self._tensors(g0.t, g0.phi, g0.psi)
        self.m = [torch.empty_like(p) for _, p in self.params]
        self.v = [torch.empty_like(p) for _, p in self.params]
        for b in self.m + self.v:
            gs3.gs3_grads_clear(b)
        self.steps_taken = [0] * len(self.params)
        self._ws: Dict[Tuple[int, int, int], Tuple[torch.Tensor, torch.Tensor, torch.Tensor]] = {}
        dev = scene.t["mean"].device
        self.loss_parts = torch.empty(2, 64, device=dev)

    @staticmethod
    def _tensors(t, phi, psi) -> List[Tuple[str, torch.Tensor]]:
        out = list(t.items())
        for m in (phi, psi):
            if m is not None:
                for w, b in m:
                    out += [("mlp", w), ("mlp", b)]
        return out

    def stage(self) -> int:
        return 1 if self.it < self.stage1_iters else 2

    def _loss_ws(self, lane: int, w: int, h: int):
        """A lane's dL/dfinal and loss workspaces (lanes run concurrently)."""
        key = (lane, w, h)
        if key not in self._ws:
            dev = self.scene.t["mean"].device
            self._ws[key] = (torch.empty(3, h, w, device=dev), gs3.l1_workspace(3 * w * h),
                             gs3.dssim_workspace(3, h, w))
        return self._ws[key]

    def step(self, batch: Sequence[Tuple[object, object, torch.Tensor]]) -> torch.Tensor:
        """One optimisation step over `batch` = [(camera, light, target
        [3, H, W])]; returns the device tensor [2, len(batch)] of each view's
        L1 and D-SSIM terms (already weighted, summing to the loss)."""
        if len(batch) > self.loss_parts.shape[1]:
            raise ValueError("at most 64 views per step")
        lambertian = self.stage() == 1
        self.scene.k = 0 if lambertian else self.k_full
        main = torch.cuda.current_stream()
        for j in range(self.lanes):
            self.streams[j].wait_stream(main)
            with torch.cuda.stream(self.streams[j]):
                self.grads[j].zero_()
                for v in range(j, len(batch), self.lanes):
                    cam, light, target = batch[v]
                    out = self.rnds[j].render(cam, light, check=False, overlap=False)
                    dF, l1ws, sws = self._loss_ws(j, cam.width, cam.height)
                    px = 3 * cam.width * cam.height * len(batch)
                    gs3.gs3_l1_loss(out["final"], target, (1.0 - self.lam) / px, self.loss_parts[0, v:v + 1], dF,
                                    l1ws)
                    gs3.gs3_dssim_loss(out["final"], target, self.lam / px, self.loss_parts[1, v:v + 1], dF, sws,
                                       accumulate=True)
                    self.rnds[j].backward(cam, light, dF, self.grads[j])
        for j in range(self.lanes):
            main.wait_stream(self.streams[j])
        for g in self.grads[1:]:
            self.grads[0].add_(g)
        for i, ((name, p), (_, g)) in enumerate(zip(self.params, self.gtens)):
            if lambertian and name in LOBES:
                continue
            self.steps_taken[i] += 1
            lr = lobe_lr(self.it) if name in LOBE_SHAPE else self.lr[name]
            gs3.gs3_adam_step(p, g, self.m[i], self.v[i], self.steps_taken[i], lr)
        self.it += 1
        return self.loss_parts[:, :len(batch)]

    def check_capacity(self, views: Sequence[Tuple[object, object]]):
        """Size every lane's buffers for these views (host syncs)."""
        for j in range(self.lanes):
            with torch.cuda.stream(self.streams[j]):
                for cam, light in views:
                    self.rnds[j].render(cam, light, check=True)
        torch.cuda.synchronize()

    def overflowed(self) -> bool:
        return any(r.overflowed() for r in self.rnds)
