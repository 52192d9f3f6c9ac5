"""gs3_l1_loss_noalloc (the L1 loss for callers that cannot allocate) against
gs3_l1_loss, called through the C-ABI: the same loss bits and the same
gradient on two calls in a row, the second with a smaller input (the
library's scratch keeps the first call's partial sums, which the second must
not read), plus the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _inputs(count, seed):
    rng = np.random.default_rng(seed)
    pred = rng.normal(0.5, 0.3, count).astype(np.float32)
    target = (pred + rng.normal(0.0, 0.05, count)).astype(np.float32)
    tie = rng.random(count) < 0.01
    target[tie] = pred[tie]              # equal elements: gradient 0
    return torch.as_tensor(pred).cuda(), torch.as_tensor(target).cuda()


def _call_both(g, pred, target, scale):
    lib = g._lib
    count = pred.numel()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ws = g.l1_workspace(count)
    wsp, wsb = g._aligned(ws)
    ref_loss = torch.full((1,), float("nan"), device="cuda")
    ref_grad = torch.full((count,), float("nan"), device="cuda")
    st = lib.gs3_l1_loss(C.c_void_p(pred.data_ptr()), C.c_void_p(target.data_ptr()), count, C.c_float(scale),
                         C.c_void_p(ref_loss.data_ptr()), C.c_void_p(ref_grad.data_ptr()), wsp, wsb, stream)
    assert st == 0, lib.gs3_last_error()
    loss = torch.full((1,), float("nan"), device="cuda")
    grad = torch.full((count,), float("nan"), device="cuda")
    st = lib.gs3_l1_loss_noalloc(C.c_void_p(pred.data_ptr()), C.c_void_p(target.data_ptr()), count,
                                 C.c_float(scale), C.c_void_p(loss.data_ptr()), C.c_void_p(grad.data_ptr()), stream)
    assert st == 0, lib.gs3_last_error()
    torch.cuda.synchronize()
    return ref_loss, ref_grad, loss, grad


def test_noalloc_matches_the_workspace_entry_point():
    assert torch.cuda.is_available()
    from paper_2410_11419_amd import gs3 as g
    # first call: 3,000,000 elements (367 chunks); second: 20,000 (3 chunks)
    for count, seed in ((3_000_000, 1), (20_000, 2)):
        pred, target = _inputs(count, seed)
        scale = 1.0 / count
        ref_loss, ref_grad, loss, grad = _call_both(g, pred, target, scale)
        print(f"[noalloc {count}] loss {loss.item():.9g} workspace entry point {ref_loss.item():.9g}")
        assert loss.cpu().numpy().view(np.uint32)[0] == ref_loss.cpu().numpy().view(np.uint32)[0]
        assert torch.equal(grad, ref_grad)
        # and the value itself: float64 sum of the float32 differences
        d = (pred.double() - target.double()).abs().sum().item() * scale
        assert abs(loss.item() - d) <= 2e-7 * abs(d)


def test_noalloc_rejects_counts_beyond_its_scratch():
    from paper_2410_11419_amd import gs3 as g
    p = C.c_void_p(256)
    st = g._lib.gs3_l1_loss_noalloc(p, p, 4096 * 8192 + 1, C.c_float(1.0), p, None, None)
    assert st == g.GS3_INVALID_ARG
    assert b"33554432" in g._lib.gs3_last_error()
