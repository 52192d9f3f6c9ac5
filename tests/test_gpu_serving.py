"""GPU tests of the continuous-batching server: overlapping requests of
mixed resolution give the same images as each request rendered alone
(1e-4 max abs; the shadow numerator's float atomics may add in another
order), requests really overlap on the device, and the memory cap bounds
the buffers the server allocates."""
import numpy as np
import pytest
import torch

from paper_2410_11419_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2410_11419_amd import gs3, serve
    assert gs3.device_ok()
    sc = synth.make_scene(40000, 8, seed=11, means="shell", mlps=True)
    return gs3, serve, gs3.DeviceScene.from_host(sc)


def test_served_equals_alone(env):
    gs3, serve, ds = env
    reqs = serve.make_requests(24, qps=1e6, seed=5, resolutions=(96, 160, 256), light_res=256)
    srv = serve.Server(ds, mem_cap_bytes=4 << 30, light_res=256, max_inflight=6)
    got = srv.run(reqs, keep_results=True)
    # real overlap: some request started before another one finished
    spans = sorted((r.start, r.done) for r in got)
    overlap = max(sum(1 for s, d in spans if s <= t < d) for t, _ in spans)
    print(f"max requests in flight together: {overlap}, buffer sets {len(srv.sets)}")
    assert overlap >= 2
    rnd = gs3.Renderer(ds)
    worst = 0.0
    for req, res in zip(reqs, got):
        alone = rnd.render(req.cam, req.light)["final"]
        assert res.final.shape == alone.shape
        worst = max(worst, float((res.final - alone).abs().max()))
    print(f"max |served - alone| = {worst:.2e}")
    assert worst <= 1e-4


def test_plain_baseline_and_memory_cap(env):
    gs3, serve, ds = env
    reqs = serve.make_requests(12, qps=2000.0, seed=6, resolutions=(64, 128), light_res=128)
    plain = serve.run_plain(ds, reqs, light_res=128, keep_results=True)
    # cap of one buffer set: the server still serves everything, one at a time
    one = serve.BufferSet(ds, gs3.default_consts(), 128, 128, max(1 << 16, 32 * ds.n)).bytes
    srv = serve.Server(ds, mem_cap_bytes=one, light_res=128)
    got = srv.run(reqs, keep_results=True)
    assert srv.allocated <= one and len(srv.sets) == 1
    for a, b in zip(plain, got):
        assert float((a.final - b.final).abs().max()) <= 1e-4
    s = serve.summarize(got)
    assert s["requests"] == 12 and s["p99_ms"] >= s["p50_ms"] > 0
