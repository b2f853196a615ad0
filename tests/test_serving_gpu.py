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


def test_auto_precision_picks_split_fp16_at_512_columns(env):
    """precision="auto" serves the 256-element array (512 columns) in split FP16 and the others
    in FP32; split FP16 on that grid meets the FP32 tolerances against the FP64 oracle (1e-5 on
    the image, 1e-4 on the NNCC): 256 elements at 0.2 mm, 1024 samples, 21 depths."""
    torch, pam, serving, pool = env
    from oracle import as_tax as O
    from paper_2412_02413_amd import synth
    srv = serving.Server(precision="auto", max_samples=1024)
    try:
        assert srv.precision_for(serving.ArrayKey(256, 40e6)) == "split_fp16"
        assert srv.precision_for(serving.ArrayKey(128, 40e6)) == "fp32"
        assert srv.precision_for(serving.ArrayKey(64, 20e6)) == "fp32"
    finally:
        srv.close()
    g = synth.cfg5_geometry(256, 40e6, 1024)
    g = g.replace(depths_m=g.depths_m[::48][:21])
    rng = np.random.default_rng(512)
    em = synth._random_emitters(rng, 3, (-20, 20), (20, 60), [])
    rf = synth.render(g, em, rng, n_t=1024, snr_db=20.0)
    plan = pam.pam_plan(g, 0, "split_fp16")
    try:
        out = pam.reconstruct(plan, torch.from_numpy(rf[None]).cuda())
        torch.cuda.synchronize()
        img, rho = out["image"][0].cpu().numpy(), out["nncc"][0].cpu().numpy()
    finally:
        pam.pam_destroy(plan)
    ref = O.as_tax(rf, g)
    e_i = float(np.linalg.norm(img - ref["I"]) / np.linalg.norm(ref["I"]))
    e_r = float(np.abs(rho - ref["rho_n"]).max())
    print(f"split FP16, 512 columns: relL2(I)={e_i:.2e} max|d rho_n|={e_r:.2e}", flush=True)
    assert e_i <= 1e-5 and e_r <= 1e-4
