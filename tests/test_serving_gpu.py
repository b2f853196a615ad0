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

