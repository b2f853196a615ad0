"""Split-precision forms of the inverse lateral transform against the FP64 oracle.

Tolerances: split BF16 / split FP16 (three 16-bit products, FP32 accumulation):
relative L2 error of the image <= 1e-3 and absolute NNCC error <= 1e-3.  The
single-product BF16 / FP16 forms are reported; they are held to a looser
bound (1e-2 on the image, 5e-2 on the NNCC) that only guards against gross
failure: a single 16-bit product does not reach 1e-3 on the NNCC.
"""
import numpy as np
import pytest

from oracle import as_tax as O
from paper_2412_02413_amd import synth

pytestmark = pytest.mark.gpu
MM = 1e-3
BOUND = {"split_bf16": (1e-3, 1e-3), "split_fp16": (1e-3, 1e-3), "bf16": (1e-2, 5e-2), "fp16": (1e-2, 5e-2)}


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2412_02413_amd import pam
    assert torch.cuda.is_available()
    pam._lib()
    return torch, pam


def gpu_run(env, geom, rf, precision):
    torch, pam = env
    plan = pam.pam_plan(geom, 0, precision)
    try:
        x = torch.from_numpy(np.ascontiguousarray(rf, np.float32)).cuda()
        out = pam.reconstruct(plan, x, want_nncc=True)
        torch.cuda.synchronize()
        return out["image"].cpu().numpy(), out["nncc"].cpu().numpy()
    finally:
        pam.pam_destroy(plan)


def errors(img, rho, ref):
    e_i = float(np.linalg.norm(img - ref["I"]) / np.linalg.norm(ref["I"]))
    e_r = float(np.abs(rho - ref["rho_n"]).max())
    return e_i, e_r


@pytest.fixture(scope="module")
def cfg1_refs():
    g = synth.cfg1_geometry()
    rf = synth.batch(synth.cfg1_frame, [40, 41])
    return g, rf, [O.as_tax(rf[f], g) for f in range(2)]


@pytest.mark.parametrize("precision", ["split_bf16", "split_fp16", "bf16", "fp16"])
def test_precision_cfg1(env, cfg1_refs, precision):
    g, rf, refs = cfg1_refs
    img, rho = gpu_run(env, g, rf, precision)
    tol_i, tol_r = BOUND[precision]
    for f in range(2):
        e_i, e_r = errors(img[f], rho[f], refs[f])
        print(f"{precision}: frame {f} relL2(I)={e_i:.3e} max|d rho_n|={e_r:.3e}", flush=True)
        assert e_i <= tol_i and e_r <= tol_r


@pytest.mark.parametrize("precision", ["split_bf16", "split_fp16"])
def test_precision_cfg2_reduced(env, precision):
    g = synth.cfg2_geometry()
    g = g.replace(depths_m=g.depths_m[np.linspace(0, 511, 40).astype(int)])
    rf, _ = synth.cfg2_frame(6)
    img, rho = gpu_run(env, g, rf[None], precision)
    e_i, e_r = errors(img[0], rho[0], O.as_tax(rf, g))
    print(f"{precision} cfg2: relL2(I)={e_i:.3e} max|d rho_n|={e_r:.3e}", flush=True)
    assert e_i <= 1e-3 and e_r <= 1e-3


def test_mixed_record_lengths_on_one_plan(env):
    """64 frames of the cfg1 array with record lengths drawn from {2048, 4096, 8192} on one
    8192-sample plan, one launch per record length.  Every form is checked against the
    FP64 oracle on the first frame of each length (FP32: 1e-5 / 1e-4; split BF16 and split
    FP16: 1e-3 / 1e-3), and the split forms against the FP32 path on every frame."""
    torch, pam = env
    g = synth.cfg3_geometry()
    frames = [synth.cfg3_frame(s) for s in range(64)]
    lengths = sorted({fr.shape[-1] for fr in frames})
    assert len(lengths) >= 2
    for n_t in lengths:
        idx = [i for i, fr in enumerate(frames) if fr.shape[-1] == n_t]
        rf = np.stack([frames[i] for i in idx])
        ref = O.as_tax(rf[0], g.replace(n_samples=n_t))
        img32, rho32 = gpu_run(env, g, rf, "fp32")
        e_i, e_r = errors(img32[0], rho32[0], ref)
        print(f"n_t={n_t} ({len(idx)} frames): fp32 vs oracle relL2(I)={e_i:.3e} max|d rho_n|={e_r:.3e}",
              flush=True)
        assert e_i <= 1e-5 and e_r <= 1e-4
        for prec in ("split_bf16", "split_fp16"):
            img, rho = gpu_run(env, g, rf, prec)
            e_i, e_r = errors(img[0], rho[0], ref)
            print(f"n_t={n_t}: {prec} vs oracle relL2(I)={e_i:.3e} max|d rho_n|={e_r:.3e}", flush=True)
            assert e_i <= 1e-3 and e_r <= 1e-3
            for k in range(len(idx)):
                e = float(np.linalg.norm(img[k] - img32[k]) / np.linalg.norm(img32[k]))
                assert e <= 1e-3 and float(np.abs(rho[k] - rho32[k]).max()) <= 1e-3


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_grouped_call_mixes_record_lengths(env, precision):
    """The 64 mixed-length frames of the cfg1 array in ONE call (groups of 2048 / 4096 / 8192
    samples back to back, with an empty group in between): every frame equals the per-length
    call on the same frames up to summation order, and the first frame of each length
    matches the FP64 oracle at the form's tolerance.  In FP32 the fields stage is one grouped
    work-list launch over all lengths when its cost estimate beats per-length launches (not
    for these 64 frames: each length fills the device on its own)."""
    torch, pam = env
    g = synth.cfg3_geometry()
    frames = [synth.cfg3_frame(s) for s in range(64)]
    lengths = sorted({fr.shape[-1] for fr in frames})
    order = {n: [i for i, fr in enumerate(frames) if fr.shape[-1] == n] for n in lengths}
    groups = [(lengths[0], len(order[lengths[0]])), (lengths[1], 0)] + [(n, len(order[n])) for n in lengths[1:]]
    packed = np.concatenate([np.stack([frames[i] for i in order[n]]).ravel() for n in lengths]).astype(np.float32)
    plan = pam.pam_plan(g, 0, precision)
    try:
        F = sum(f for _, f in groups)
        rf = torch.from_numpy(packed).cuda()
        img = torch.empty((F, g.n_z, g.n_x), device="cuda")
        rho = torch.empty_like(img)
        ws = pam.alloc_workspace_grouped(plan, groups)
        assert not pam.debug_grouped_one_launch(plan, groups)
        pam.pam_as_tax_grouped(plan, rf, groups, img, rho, None, ws)
        torch.cuda.synchronize()
        img, rho = img.cpu().numpy().astype(np.float64), rho.cpu().numpy().astype(np.float64)
        with pytest.raises(pam.PamError):
            pam.pam_workspace_size_grouped(plan, [(1000, 3)])                 # not a record length of the plan
        with pytest.raises(pam.PamError):
            pam.pam_workspace_size_grouped(plan, [(lengths[0], 1)] * 9)       # more than 8 groups
    finally:
        pam.pam_destroy(plan)
    tol_i, tol_r = (1e-5, 1e-4) if precision == "fp32" else (1e-3, 1e-3)
    k = 0
    for n in lengths:
        idx = order[n]
        alone_i, alone_r = gpu_run(env, g, np.stack([frames[i] for i in idx]), precision)
        for j in range(len(idx)):
            e = float(np.linalg.norm(img[k + j] - alone_i[j]) / np.linalg.norm(alone_i[j]))
            assert e <= 1e-5 and float(np.abs(rho[k + j] - alone_r[j]).max()) <= 1e-4, (n, j, e)
        ref = O.as_tax(frames[idx[0]], g.replace(n_samples=n))
        e_i, e_r = errors(img[k], rho[k], ref)
        print(f"{precision} n_t={n} ({len(idx)} frames): grouped vs oracle relL2(I)={e_i:.3e} "
              f"max|d rho_n|={e_r:.3e}", flush=True)
        assert e_i <= tol_i and e_r <= tol_r
        k += len(idx)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_grouped_work_list_launch(env, precision):
    """One frame of each record length on a shallow grid (33 depths: two depth tiles a frame
    at 128 columns in FP32): no length fills the device alone, so the fields stage runs as ONE
    grouped work-list launch (FP32; the split form at 128 columns runs per length).  An empty
    group sits between the first two, so the work list also skips a zero-frame group.  Every
    frame equals its per-length call up to summation order and the FP64 oracle at the form's
    tolerance."""
    torch, pam = env
    g = synth.cfg3_geometry().replace(depths_m=(20 + 0.5 * np.arange(33)) * MM)
    rng = np.random.default_rng(21)
    em = [synth.Emitter(1 * MM, 30 * MM, "broadband"), synth.Emitter(-4 * MM, 26 * MM, "stable")]
    lengths = [2048, 4096, 8192]
    frames = {n: synth.render(g, em, rng, n_t=n)[None] for n in lengths}
    groups = [(lengths[0], 1), (lengths[1], 0)] + [(n, 1) for n in lengths[1:]]
    plan = pam.pam_plan(g, 0, precision)
    try:
        assert pam.debug_grouped_one_launch(plan, groups) == (precision == "fp32")
        rf = torch.from_numpy(np.concatenate([frames[n].ravel() for n in lengths]).astype(np.float32)).cuda()
        img = torch.empty((3, g.n_z, g.n_x), device="cuda")
        rho = torch.empty_like(img)
        ws = pam.alloc_workspace_grouped(plan, groups)
        pam.pam_as_tax_grouped(plan, rf, groups, img, rho, None, ws)
        torch.cuda.synchronize()
        img, rho = img.cpu().numpy().astype(np.float64), rho.cpu().numpy().astype(np.float64)
    finally:
        pam.pam_destroy(plan)
    tol_i, tol_r = (1e-5, 1e-4) if precision == "fp32" else (1e-3, 1e-3)
    for k, n in enumerate(lengths):
        alone_i, alone_r = gpu_run(env, g, frames[n], precision)
        e = float(np.linalg.norm(img[k] - alone_i[0]) / np.linalg.norm(alone_i[0]))
        assert e <= 1e-5 and float(np.abs(rho[k] - alone_r[0]).max()) <= 1e-4, (n, e)
        e_i, e_r = errors(img[k], rho[k], O.as_tax(frames[n][0], g.replace(n_samples=n)))
        print(f"{precision} n_t={n}: grouped vs oracle relL2(I)={e_i:.3e} max|d rho_n|={e_r:.3e}", flush=True)
        assert e_i <= tol_i and e_r <= tol_r
