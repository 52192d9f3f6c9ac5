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


def test_served_equals_alone_at_serving_workload(env):
    """The serving workload's own scene and sizes: 300,000 Gaussians,
    camera 256^2 / 512^2 / 800^2 / 1024^2, light 1024^2; 16 requests arriving
    at once, up to 8 in flight, each result equal to the request rendered
    alone."""
    gs3, serve, _ = env
    sc, _, _ = synth.scene_full()
    ds = gs3.DeviceScene.from_host(sc)
    reqs = serve.make_requests(16, qps=1e6, seed=8)
    assert {r.cam.width for r in reqs} == {256, 512, 800, 1024}
    srv = serve.Server(ds, mem_cap_bytes=24 << 30, max_inflight=8)
    got = srv.run(reqs, keep_results=True)
    spans = sorted((r.start, r.done) for r in got)
    overlap = max(sum(1 for s, d in spans if s <= t < d) for t, _ in spans)
    rnd = gs3.Renderer(ds)
    worst = 0.0
    for req, res in zip(reqs, got):
        alone = rnd.render(req.cam, req.light)["final"]
        assert res.final.shape == alone.shape
        worst = max(worst, float((res.final - alone).abs().max()))
    print(f"300K scene: max requests in flight together {overlap}, max |served - alone| = {worst:.2e}")
    assert overlap >= 2
    assert worst <= 1e-4


def test_memory_cap_with_mixed_resolutions(env):
    """Requests of 64^2 and 256^2 under a cap that holds one small and one
    large set at most: the server never allocates past the cap, and frees
    idle sets of the other resolution to make room."""
    gs3, serve, ds = env
    cap_small = serve.BufferSet.estimate(ds.n, 64, 128, max(1 << 16, 32 * ds.n))
    cap_large = serve.BufferSet.estimate(ds.n, 256, 128, max(1 << 16, 32 * ds.n))
    cap = cap_small + cap_large + 1
    reqs = serve.make_requests(20, qps=3000.0, seed=7, resolutions=(64, 256), light_res=128)
    srv = serve.Server(ds, mem_cap_bytes=cap, light_res=128, max_inflight=4)
    peak = 0
    orig = srv._acquire

    def watch(res):
        nonlocal peak
        bs = orig(res)
        peak = max(peak, srv.allocated)
        return bs
    srv._acquire = watch
    got = srv.run(reqs, keep_results=True)
    print(f"cap {cap} bytes, peak allocated {peak}, sets {len(srv.sets)}")
    assert peak <= cap and srv.allocated <= cap
    assert all(r.final is not None for r in got)


def test_shared_lights_equal_alone(env):
    """Light sharing: 24 requests of mixed resolution under 3 distinct
    lights run 3 shadow passes, and every result equals the request
    rendered alone."""
    gs3, serve, ds = env
    reqs = serve.make_requests(24, qps=1e6, seed=12, resolutions=(96, 160, 256), light_res=256, n_lights=3)
    assert len({serve.light_key(r.light) for r in reqs}) == 3
    srv = serve.Server(ds, mem_cap_bytes=4 << 30, light_res=256, max_inflight=6, share_lights=True)
    got = srv.run(reqs, keep_results=True)
    rnd = gs3.Renderer(ds)
    worst = 0.0
    for req, res in zip(reqs, got):
        alone = rnd.render(req.cam, req.light)["final"]
        worst = max(worst, float((res.final - alone).abs().max()))
    print(f"shadow passes {srv.light_passes} for 24 requests, max |served - alone| = {worst:.2e}")
    assert srv.light_passes == 3
    assert worst <= 1e-4


def test_batched_server_equals_alone(env):
    """Batched launches: 24 requests arriving at once, mixed resolutions,
    batches of up to 6 requests per launch sequence; every result equals the
    request rendered alone, and fewer launch sequences than requests ran."""
    gs3, serve, ds = env
    reqs = serve.make_requests(24, qps=1e6, seed=9, resolutions=(96, 160, 256), light_res=256)
    srv = serve.Server(ds, mem_cap_bytes=4 << 30, light_res=256, max_inflight=12, batch=6)
    got = srv.run(reqs, keep_results=True)
    rnd = gs3.Renderer(ds)
    worst = 0.0
    for req, res in zip(reqs, got):
        alone = rnd.render(req.cam, req.light)["final"]
        assert res.final.shape == alone.shape
        worst = max(worst, float((res.final - alone).abs().max()))
    print(f"batches {srv.batches} for 24 requests, max |served - alone| = {worst:.2e}")
    assert srv.batches < 24
    assert worst <= 1e-4


def test_batched_server_at_serving_workload(env):
    """The serving workload's scene and sizes (300,000 Gaussians, cameras
    256^2 to 1024^2, light 1024^2), 16 requests at once in batches of up to
    8, shared lights within a batch: each result equals the request alone."""
    gs3, serve, _ = env
    sc, _, _ = synth.scene_full()
    ds = gs3.DeviceScene.from_host(sc)
    reqs = serve.make_requests(16, qps=1e6, seed=8, n_lights=5)
    srv = serve.Server(ds, mem_cap_bytes=24 << 30, max_inflight=16, batch=8, share_lights=True)
    got = srv.run(reqs, keep_results=True)
    rnd = gs3.Renderer(ds)
    worst = 0.0
    for req, res in zip(reqs, got):
        alone = rnd.render(req.cam, req.light)["final"]
        worst = max(worst, float((res.final - alone).abs().max()))
    print(f"300K scene: batches {srv.batches}, shadow passes {srv.light_passes}, max |served - alone| = {worst:.2e}")
    assert srv.batches < 16 and srv.light_passes <= 5
    assert worst <= 1e-4
