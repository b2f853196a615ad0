"""Continuous-batching server: results in the mix equal results alone, HBM-budget
admission, and requests admitted while other batches are on the GPU."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2412_02413_amd import pam, serving
    assert torch.cuda.is_available()
    pam._lib()
    pool = serving.make_pool(seed=3, arrays=(64, 128), rates=(20e6, 40e6), lengths=(1024, 2048))
    return torch, pam, serving, pool


def alone(pam, torch, srv, req):
    p = srv.plan(req.key)
    rf = req.rf.to(srv.device)[None]
    out = pam.reconstruct(p, rf, want_nncc=False)
    torch.cuda.synchronize()
    return out["image"][0].cpu().numpy()


def test_mix_equals_alone(env):
    torch, pam, serving, pool = env
    srv = serving.Server(max_batch=8, n_streams=3, max_samples=2048)
    try:
        reqs = serving.poisson_requests(pool, 20000.0, 40, seed=5)
        srv.run(reqs)
        assert all(r.status == "done" for r in reqs)
        assert srv.stats["max_inflight"] >= 2          # batches overlapped on the device
        assert max(srv.batch_sizes) >= 2               # requests were batched
        for r in reqs[:12]:
            ref = alone(pam, torch, srv, r)
            e = float(np.linalg.norm(r.image - ref) / np.linalg.norm(ref))
            assert e <= 1e-5, (r.rid, e)
    finally:
        srv.close()


def test_largest_frame_in_the_mix_equals_alone(env):
    """The largest serving frame, a 256-element array on 512 columns with 16,384 samples at
    40 MHz, served in a mix with small 64-element requests: each of its images equals the same
    request run alone (relative L2 1e-5; only the bin split of the batch changes the FP32
    summation order)."""
    torch, pam, serving, _ = env
    pool = serving.make_pool(seed=11, arrays=(64, 256), rates=(40e6,), lengths=(1024, 16384))
    srv = serving.Server(max_batch=4, n_streams=3, max_samples=16384)
    try:
        reqs = serving.poisson_requests(pool, 5000.0, 16, seed=7)
        big = [r for r in reqs if r.key.n_elements == 256 and r.n_t == 16384]
        assert big, "the request mix holds no 256-element, 16,384-sample frame"
        srv.run(reqs)
        assert all(r.status == "done" for r in reqs)
        for r in big[:3]:
            ref = alone(pam, torch, srv, r)
            e = float(np.linalg.norm(r.image - ref) / np.linalg.norm(ref))
            print(f"request {r.rid}: 256 elements, 16384 samples, mixed vs alone relL2 {e:.2e}", flush=True)
            assert e <= 1e-5, (r.rid, e)
    finally:
        srv.close()


def test_budget_admission_and_rejection(env):
    torch, pam, serving, pool = env
    probe = serving.Server(max_samples=2048)
    key = serving.ArrayKey(64, 20e6)
    one = probe.batch_bytes(key, 2048, 1)
    probe.close()
    # a budget that holds exactly one frame: everything completes, one batch at a time
    srv = serving.Server(max_batch=8, n_streams=3, hbm_budget=one, max_samples=2048)
    try:
        reqs = [serving.Request(i, key, 2048, pool[(key, 2048)], t_arrival=0.0) for i in range(5)]
        srv.run(reqs, realtime=False)
        assert all(r.status == "done" for r in reqs)
        assert srv.stats["max_inflight"] == 1 and max(srv.batch_sizes) == 1
    finally:
        srv.close()
    # a budget below one frame: requests are refused, nothing crashes
    srv = serving.Server(hbm_budget=one // 2, max_samples=2048)
    try:
        reqs = [serving.Request(i, key, 2048, pool[(key, 2048)], t_arrival=0.0) for i in range(3)]
        srv.run(reqs, realtime=False)
        assert all(r.status == "rejected" for r in reqs)
    finally:
        srv.close()

