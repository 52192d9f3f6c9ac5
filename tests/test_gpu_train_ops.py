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
    gs3.gs3_render(ds, cam, light, k, torch.ones(sc.n, device="cuda"), cvb, im, use_mlps=False)
    torch.cuda.synchronize()
    for key in ("final", "S", "Sh", "R", "T_final"):
        assert torch.isnan(im[key]).all(), key


@pytest.mark.parametrize("shape", [(3, 16, 16), (3, 37, 53), (1, 5, 300), (3, 800, 800)])
def test_dssim_loss_against_oracle(gs3, shape):
    """gs3_dssim_loss against the oracle's SSIM (float64, conv2d with the
    same window): the value to 2e-6 relative, the gradient to 1e-4 of its
    largest entry; accumulate adds to what the buffer holds."""
    rng = np.random.default_rng(sum(shape))
    c, h, w = shape
    base = rng.uniform(0, 1, shape)
    # smooth structure plus noise, so local statistics vary
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    base = 0.5 * base + 0.25 * (1 + np.sin(xx / 7.0 + yy / 11.0))[None]
    pred = base.astype(np.float32)
    target = np.clip(base + rng.normal(0, 0.08, shape), 0, 1).astype(np.float32)
    lam = O.LOSS_LAMBDA
    scale = lam / (c * h * w)
    p, t = torch.as_tensor(pred).cuda(), torch.as_tensor(target).cuda()
    loss = torch.zeros(1, device="cuda")
    grad = torch.full(shape, float("nan"), device="cuda")
    ws = gs3.dssim_workspace(c, h, w)
    gs3.gs3_dssim_loss(p, t, scale, loss, grad, ws)
    torch.cuda.synchronize()
    ref, gref = O.dssim_loss(pred, target, scale)
    got = float(loss.item())
    g = grad.cpu().numpy()
    gerr = float(np.abs(g - gref).max())
    gmax = float(np.abs(gref).max())
    print(f"[dssim {shape}] loss {got:.8g} oracle {ref:.8g}; grad max err {gerr:.2e} of {gmax:.2e}")
    assert abs(got - ref) <= 2e-6 * abs(ref)
    assert gerr <= 1e-4 * gmax
    # accumulate: a second call adds the same gradient
    gs3.gs3_dssim_loss(p, t, scale, loss, grad, ws, accumulate=True)
    torch.cuda.synchronize()
    assert float(np.abs(grad.cpu().numpy() - 2 * g).max()) <= 1e-6 * gmax + 1e-30


def test_adam_against_oracle(gs3):
    rng = np.random.default_rng(9)
    n = 100_003
    p0 = rng.normal(size=n).astype(np.float32)
    p, m, v = torch.as_tensor(p0).cuda(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    po, mo, vo = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 6):
        g = (rng.normal(size=n) * 10 ** rng.uniform(-6, 1, n)).astype(np.float32)
        gs3.gs3_adam_step(p, torch.as_tensor(g).cuda(), m, v, step, 0.01)
        po, mo, vo = O.adam_step(po, g, mo, vo, step, 0.01)
    torch.cuda.synchronize()
    err = float(np.abs(p.cpu().numpy() - po).max())
    print(f"[adam] 5 steps over {n} parameters: max |param err| {err:.2e}")
    assert err <= 2e-6


def test_lambertian_stage(gs3):
    """The first training stage (Sec. 4.4: appearance limited to the
    Lambertian term): a scene handed to the library with k = 0 lobes renders
    as the oracle's scene without lobes, and its backward leaves the lobe
    gradients untouched."""
    from parity_resolve import resolve
    sc = synth.make_scene(3000, 8, seed=17, means="shell", mlps=True, log_scale_mu=(-3.4,) * 3)
    rng = np.random.default_rng(17)
    cam = synth.make_view(rng.standard_normal(3), 4.0, 96, 80, 40.0)
    light = synth.make_view(rng.standard_normal(3), 4.0, 128, 128, 40.0)
    ds = gs3.DeviceScene.from_host(sc)
    ds.k = 0                                     # lobes off
    rnd = gs3.Renderer(ds)
    out = rnd.render(cam, light)
    torch.cuda.synchronize()
    lamb = synth.Scene(**{f: getattr(sc, f) for f in ("mean", "log_scale", "rot", "opacity_logit", "shade_rot",
                                                       "albedo", "feat")},
                       lobe_axis=sc.lobe_axis[:0], lobe_log_sharp=sc.lobe_log_sharp[:0], lobe_amp=sc.lobe_amp[:0],
                       phi=sc.phi, psi=sc.psi)
    npx = cam.width * cam.height
    px = {k: out[k].cpu().numpy().reshape(-1, npx).squeeze(0) if out[k].dim() == 2 else
          out[k].cpu().numpy().reshape(3, npx) for k in ("final", "S", "Sh", "R", "T_final")}
    ref, info = resolve(lamb, cam, light, O.Consts(), sc.phi.layers, sc.psi.layers, out["T"].cpu().numpy()[:sc.n], px)
    err = float(np.abs(out["final"].cpu().numpy().reshape(3, -1) - ref["final"].detach().numpy()).max())
    errc = float(np.abs(out["colour"].cpu().numpy()[0:3, :sc.n] - ref["c"].detach().numpy().T).max())
    print(f"[lambertian] final err {err:.2e}, colour err {errc:.2e}")
    assert err <= 1e-4 and errc <= 1e-4
    dF = torch.randn(3, cam.height, cam.width, generator=torch.Generator().manual_seed(1)).cuda() / 100
    g = rnd.backward(cam, light, dF)
    torch.cuda.synchronize()
    for nm in ("lobe_axis", "lobe_log_sharp", "lobe_amp"):
        assert float(g.t[nm].abs().max()) == 0.0, nm
    assert float(g.t["albedo"].abs().max()) > 0


def test_trainer_step_against_oracle(gs3):
    """One optimisation step of the full objective (Sec. 4.4): two views on
    two lanes, loss (1 - lambda) L1 + lambda D-SSIM, the first (Lambertian)
    stage. Checked against the oracle: each view's two loss terms, the
    batch gradient of every raw parameter and MLP weight (float64 autograd
    of the oracle's render with the GPU's float32-ambiguous decisions, the
    L1 subgradient and the SSIM), no update of the lobes, and every other
    tensor moved by one Adam step from the GPU's own gradient."""
    from parity_resolve import resolve
    from paper_2410_11419_amd import train
    sc = synth.make_scene(2500, 4, seed=21, means="shell", mlps=True, log_scale_mu=(-3.4,) * 3)
    rng = np.random.default_rng(21)
    views = [(synth.make_view(rng.standard_normal(3), 4.0, 72, 64, 40.0),
              synth.make_view(rng.standard_normal(3), 4.0, 112, 112, 40.0)) for _ in range(2)]
    tgt = gs3.Renderer(gs3.DeviceScene.from_host(synth.perturb_scene(sc, seed=22)))
    targets = [tgt.render(c, l)["final"].clone() for c, l in views]
    ds = gs3.DeviceScene.from_host(sc)
    tr = train.Trainer(ds, lanes=2, stage1_iters=1)
    tr.check_capacity(views)
    before = [p.detach().clone() for _, p in tr.params]
    parts = tr.step([(c, l, t) for (c, l), t in zip(views, targets)]).cpu().numpy()
    torch.cuda.synchronize()
    g_gpu = [g.cpu().numpy() for _, g in tr.gtens]
    # the oracle: the Lambertian scene (no lobes), both views' renders with
    # the GPU's ambiguous decisions, one float64 loss for the batch
    lamb = synth.Scene(**{f: getattr(sc, f) for f in ("mean", "log_scale", "rot", "opacity_logit", "shade_rot",
                                                       "albedo", "feat")},
                       lobe_axis=sc.lobe_axis[:0], lobe_log_sharp=sc.lobe_log_sharp[:0], lobe_amp=sc.lobe_amp[:0],
                       phi=sc.phi, psi=sc.psi)
    p = O.scene_tensors(lamb, requires_grad=True)
    mlp = lambda L: [(torch.tensor(w, dtype=torch.float64, requires_grad=True),  # noqa: E731
                      torch.tensor(b, dtype=torch.float64, requires_grad=True)) for w, b in L]
    phi, psi = mlp(sc.phi.layers), mlp(sc.psi.layers)
    total = 0.0
    px_all = sum(3 * c.width * c.height for c, _ in views)
    for j, ((cam, light), target) in enumerate(zip(views, targets)):
        r = tr.rnds[j]
        out = r._images(cam.width, cam.height)
        npx = cam.width * cam.height
        px = {k: out[k].cpu().numpy().reshape(-1, npx).squeeze(0) if out[k].dim() == 2 else
              out[k].cpu().numpy().reshape(3, npx) for k in ("final", "S", "Sh", "R", "T_final")}
        ref, _ = resolve(lamb, cam, light, O.Consts(), phi, psi, r.T.cpu().numpy()[:sc.n], px, params=p)
        f = ref["final"].reshape(3, cam.height, cam.width)
        t = torch.as_tensor(target.cpu().numpy(), dtype=torch.float64)
        l1 = (1 - O.LOSS_LAMBDA) * (f - t).abs().sum() / px_all
        ds_ = O.LOSS_LAMBDA * (1 - O.ssim_map(f, t)).sum() / px_all
        print(f"[trainer] view {j}: L1 term {parts[0, j]:.8g} oracle {float(l1):.8g}; D-SSIM term "
              f"{parts[1, j]:.8g} oracle {float(ds_):.8g}")
        assert abs(parts[0, j] - float(l1)) <= 1e-5 * float(l1)
        assert abs(parts[1, j] - float(ds_)) <= 1e-5 * float(ds_)
        total = total + l1 + ds_
    total.backward()
    ref_g = [p[nm].grad for nm in gs3.SCENE_FIELDS if nm not in train.LOBES]
    ref_g += [x.grad for m in (phi, psi) for pair in m for x in pair]
    names = [nm for nm, _ in tr.params]
    got = [g for (nm, _), g in zip(tr.params, g_gpu) if nm not in train.LOBES]
    to_lib = {"mean": lambda x: x.T, "log_scale": lambda x: x.T, "rot": lambda x: x.T, "opacity_logit": lambda x: x,
              "shade_rot": lambda x: x.T, "albedo": lambda x: x.T, "feat": lambda x: x.T}
    worst = 0.0
    for nm, a, rg in zip([n for n in names if n not in train.LOBES], got, ref_g):
        r_ = (to_lib[nm](rg) if nm in to_lib else rg).numpy()
        # the loss is a mean over every pixel of the batch, so gradients are
        # small: compare relative to each tensor's largest entry
        scale = max(1e-12, float(np.abs(r_).max()))
        e = float(np.abs(a - r_).max()) / scale
        worst = max(worst, e)
        assert e <= 1e-3, (nm, e)
    print(f"[trainer] gradient error relative to each tensor's largest entry: {worst:.1e}")
    # the update: lobes untouched in the first stage; every other tensor one
    # Adam step (lr of its group) from the GPU gradient
    for i, (nm, p_after) in enumerate(tr.params):
        pa = p_after.cpu().numpy()
        if nm in train.LOBES:
            assert np.array_equal(pa, before[i].cpu().numpy()), nm
            continue
        lr = tr.lr[nm]
        want, _, _ = O.adam_step(before[i].cpu().numpy(), g_gpu[i], 0.0, 0.0, 1, lr)
        assert float(np.abs(pa - want).max()) <= 1e-6 * max(1.0, float(np.abs(want).max())), nm
    assert tr.stage() == 2 and tr.it == 1


def test_trainer_step_basis_appearance(gs3):
    """One optimisation step of the full objective in the second stage for a
    scene with the paper's shared-basis appearance: loss terms, every
    gradient (scene, latent, shared basis, both MLPs) and one Adam update of
    every tensor, against the oracle."""
    from parity_resolve import resolve
    from paper_2410_11419_amd import train
    sc = synth.make_basis_scene(2000, 23, k=4, means="shell", mlps=True, log_scale_mu=(-3.4,) * 3)
    rng = np.random.default_rng(23)
    views = [(synth.make_view(rng.standard_normal(3), 4.0, 64, 56, 40.0),
              synth.make_view(rng.standard_normal(3), 4.0, 96, 96, 40.0)) for _ in range(2)]
    tgt = gs3.Renderer(gs3.DeviceScene.from_host(synth.perturb_scene(sc, seed=24)))
    targets = [tgt.render(c, l)["final"].clone() for c, l in views]
    ds = gs3.DeviceScene.from_host(sc)
    tr = train.Trainer(ds, lanes=2, stage1_iters=0)
    tr.check_capacity(views)
    before = [p.detach().clone() for _, p in tr.params]
    parts = tr.step([(c, l, t) for (c, l), t in zip(views, targets)]).cpu().numpy()
    torch.cuda.synchronize()
    g_gpu = [g.cpu().numpy() for _, g in tr.gtens]
    p = O.scene_tensors(sc, requires_grad=True)
    mlp = lambda L: [(torch.tensor(w, dtype=torch.float64, requires_grad=True),  # noqa: E731
                      torch.tensor(b, dtype=torch.float64, requires_grad=True)) for w, b in L]
    phi, psi = mlp(sc.phi.layers), mlp(sc.psi.layers)
    total = 0.0
    px_all = sum(3 * c.width * c.height for c, _ in views)
    for j, ((cam, light), target) in enumerate(zip(views, targets)):
        r = tr.rnds[j]
        out = r._images(cam.width, cam.height)
        npx = cam.width * cam.height
        px = {k: out[k].cpu().numpy().reshape(-1, npx).squeeze(0) if out[k].dim() == 2 else
              out[k].cpu().numpy().reshape(3, npx) for k in ("final", "S", "Sh", "R", "T_final")}
        ref, _ = resolve(sc, cam, light, O.Consts(), phi, psi, r.T.cpu().numpy()[:sc.n], px, params=p)
        f = ref["final"].reshape(3, cam.height, cam.width)
        t = torch.as_tensor(target.cpu().numpy(), dtype=torch.float64)
        l1 = (1 - O.LOSS_LAMBDA) * (f - t).abs().sum() / px_all
        ds_ = O.LOSS_LAMBDA * (1 - O.ssim_map(f, t)).sum() / px_all
        assert abs(parts[0, j] - float(l1)) <= 1e-5 * float(l1)
        assert abs(parts[1, j] - float(ds_)) <= 1e-5 * float(ds_)
        total = total + l1 + ds_
    total.backward()
    ref_g = [p[nm].grad for nm in ds.t] + [x.grad for m in (phi, psi) for pair in m for x in pair]
    worst = 0.0
    for (nm, _), a, rg in zip(tr.params, g_gpu, ref_g):
        r_ = rg.numpy()
        if r_.ndim == 2 and nm not in ("basis_rot", "basis_log_sigma") and r_.shape != a.shape:
            r_ = r_.T
        assert a.shape == r_.shape, (nm, a.shape, r_.shape)
        scale = max(1e-12, float(np.abs(r_).max()))
        e = float(np.abs(a - r_).max()) / scale
        worst = max(worst, e)
        assert e <= 1e-3, (nm, e)
    print(f"[trainer basis] gradient error relative to each tensor's largest entry: {worst:.1e}")
    for i, (nm, p_after) in enumerate(tr.params):
        lr = train.lobe_lr(0) if nm in train.LOBE_SHAPE else tr.lr[nm]
        want, _, _ = O.adam_step(before[i].cpu().numpy(), g_gpu[i], 0.0, 0.0, 1, lr)
        assert float(np.abs(p_after.cpu().numpy() - want).max()) <= 1e-6 * max(1.0, float(np.abs(want).max())), nm
