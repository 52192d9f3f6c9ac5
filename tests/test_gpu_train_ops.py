"""GPU checks of the training-step kernels behind the C-ABI (Sec. 4.4) and of
the binning status block.

- gs3_l1_loss: the value against the oracle's float64 sum (float32 inputs,
  so only the float64 summation order and the final float32 rounding
  differ: 2e-7 relative), the gradient bit for bit (the sign of a float32
  difference is exact), and the same bits on every run;
- gs3_grads_clear / gs3_grads_accumulate: exact;
- an overflowed binning: reported by the status block once it has run,
  every consumer then refuses the workspace, and without a status block the
  shadow values and images come out as NaN instead of plausible values.
"""
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


@pytest.mark.parametrize("count", [0, 1, 255, 8191, 8192, 8193, 3 * 200 * 152, 4 * 3 * 800 * 800])
def test_l1_loss_against_oracle(gs3, count):
    rng = np.random.default_rng(count % 1000 + 7)
    pred = rng.normal(0.5, 0.3, count).astype(np.float32)
    target = (pred + rng.normal(0.0, 0.05, count)).astype(np.float32)
    if count > 10:
        tie = rng.random(count) < 0.01
        target[tie] = pred[tie]                      # equal elements: gradient 0
    scale = np.float32(1.0 / max(count, 1))
    p, t = torch.as_tensor(pred).cuda(), torch.as_tensor(target).cuda()
    loss = torch.full((1,), float("nan"), device="cuda")
    grad = torch.full((max(count, 1),), float("nan"), device="cuda")[:count]
    ws = gs3.l1_workspace(count)
    gs3.gs3_l1_loss(p, t, float(scale), loss, grad, ws)
    torch.cuda.synchronize()
    ref, gref = O.l1_loss(pred, target, float(scale))
    got = float(loss.item())
    print(f"[l1 {count}] loss {got:.9g} oracle {ref:.9g} rel {abs(got - ref) / max(abs(ref), 1e-30):.2e}")
    assert abs(got - ref) <= 2e-7 * abs(ref) + 1e-30
    np.testing.assert_array_equal(grad.cpu().numpy(), gref.astype(np.float32))
    # the same bits on a second run, and without the gradient
    loss2 = torch.empty(1, device="cuda")
    gs3.gs3_l1_loss(p, t, float(scale), loss2, None, ws)
    torch.cuda.synchronize()
    assert loss2.cpu().numpy().view(np.uint32)[0] == loss.cpu().numpy().view(np.uint32)[0]


def test_gradient_set_clear_and_accumulate(gs3):
    rng = np.random.default_rng(3)
    for count, offset in ((1, 0), (1001, 0), (1001, 1), (4 * 300_000 + 3, 2)):
        a = rng.normal(size=count + offset).astype(np.float32)
        b = rng.normal(size=count + offset).astype(np.float32)
        da, db = torch.as_tensor(a).cuda(), torch.as_tensor(b).cuda()
        # misaligned views exercise the scalar path
        gs3.gs3_grads_accumulate(da[offset:], db[offset:])
        torch.cuda.synchronize()
        want = a.copy()
        want[offset:] = a[offset:] + b[offset:]
        np.testing.assert_array_equal(da.cpu().numpy(), want)
        gs3.gs3_grads_clear(da[offset:])
        torch.cuda.synchronize()
        got = da.cpu().numpy()
        assert (got[offset:] == 0).all() and (got[:offset] == want[:offset]).all()


def _overflow_case(gs3, status):
    sc, cam, light = synth.scene_small()
    ds = gs3.DeviceScene.from_host(sc)
    k = gs3.default_consts()
    vb = gs3.ViewBuffer(sc.n, light.width, light.height, 2000, status=status)   # far too few pairs
    gs3.gs3_preprocess(ds, light, k, gs3.GS3_DEPTH_DIST, vb)
    return sc, cam, light, ds, k, vb


def test_overflow_reported_by_the_status_block(gs3):
    sc, cam, light, ds, k, vb = _overflow_case(gs3, True)
    torch.cuda.synchronize()
    state, req = gs3.gs3_view_poll(vb)
    p = O.scene_tensors(sc)
    cov = O.covariance(p["log_scale"], p["rot"])
    pr = O.project(p["mean"], cov, light, O.Consts(), "dist")
    ix, iy, rx, ry = O.splat_extent(pr, O.sigmoid(p["opacity_logit"]), O.Consts())
    print(f"[status] state {state}, required {req}")
    assert state == gs3.GS3_VIEW_OVERFLOW
    # the required count is the unclamped pair total (extents may differ by
    # one where the float64 extent sits on an integer, so compare loosely)
    x0, x1, y0, y1, empty = O.tile_rects(ix, iy, rx, ry, light.width, light.height)
    ref = int(((x1 - x0 + 1) * (y1 - y0 + 1))[~empty].sum())
    assert abs(req - ref) <= 0.001 * ref
    nd = torch.empty(2, sc.n, device="cuda")
    T = torch.empty(sc.n, device="cuda")
    with pytest.raises(gs3.Gs3Error) as ei:
        gs3.gs3_shadow_splat(k, vb, nd, T)
    assert ei.value.status == gs3.GS3_PAIR_CAPACITY_EXCEEDED
    # a binning with room: pending until it runs, then OK with the same count
    vb2 = gs3.ViewBuffer(sc.n, light.width, light.height, req + 100)
    gs3.gs3_preprocess(ds, light, k, gs3.GS3_DEPTH_DIST, vb2)
    torch.cuda.synchronize()
    assert gs3.gs3_view_poll(vb2) == (gs3.GS3_VIEW_OK, req)
    assert gs3.gs3_view_pair_count(vb2) == req
    gs3.gs3_shadow_splat(k, vb2, nd, T)
    torch.cuda.synchronize()
    assert torch.isfinite(T).all()
    # rebinning the first workspace: pending until it has run, then the
    # same overflow again
    gs3.gs3_preprocess(ds, light, k, gs3.GS3_DEPTH_DIST, vb)
    torch.cuda.synchronize()
    assert gs3.gs3_view_poll(vb) == (gs3.GS3_VIEW_OVERFLOW, req)


def test_overflow_without_status_block_gives_nan(gs3):
    sc, cam, light, ds, k, vb = _overflow_case(gs3, False)
    nd = torch.empty(2, sc.n, device="cuda")
    T = torch.zeros(sc.n, device="cuda")
    gs3.gs3_shadow_splat(k, vb, nd, T)
    torch.cuda.synchronize()
    assert torch.isnan(T).all()
    # the camera side: a camera binning that overflows gives NaN images
    cvb = gs3.ViewBuffer(sc.n, cam.width, cam.height, 500, status=False)
    gs3.gs3_preprocess(ds, cam, k, gs3.GS3_DEPTH_Z, cvb)
    im = {"final": torch.zeros(3, cam.height, cam.width, device="cuda"),
          "S": torch.zeros(3, cam.height, cam.width, device="cuda"),
          "Sh": torch.zeros(cam.height, cam.width, device="cuda"),
          "R": torch.zeros(3, cam.height, cam.width, device="cuda"),
          "T_final": torch.zeros(cam.height, cam.width, device="cuda"),
          "n_contrib": torch.zeros(cam.height, cam.width, dtype=torch.int32, device="cuda"),
          "colour": torch.zeros(8, sc.n, device="cuda")}
    gs3.gs3_render(ds, cam, light.eye, k, torch.ones(sc.n, device="cuda"), cvb, im, use_mlps=False)
    torch.cuda.synchronize()
    for key in ("final", "S", "Sh", "R", "T_final"):
        assert torch.isnan(im[key]).all(), key
