"""FD-TEA-TAX (pam_fd_tea_tax) against the FP64 oracle of oracle/fd_tea.py: the same
tolerances as the AS-TAX FP32 path (relative L2 of the image <= 1e-5, absolute NNCC
error <= 1e-4)."""
import numpy as np
import pytest

from oracle import fd_tea as T
from paper_2412_02413_amd import synth

pytestmark = pytest.mark.gpu
MM = 1e-3


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2412_02413_amd import pam
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pam._lib()
    return torch, pam


def gpu_fd_tea(env, geom, rf):
    torch, pam = env
    plan = pam.pam_plan(geom, 0, "fp32")
    try:
        x = torch.from_numpy(np.ascontiguousarray(rf, np.float32)).cuda()
        F = x.shape[0]
        img = torch.empty((F, plan.n_z, plan.n_x), device="cuda")
        nncc = torch.empty_like(img)
        pairs = torch.empty((F, plan.n_pairs, plan.n_z, plan.n_x), device="cuda") if plan.n_pairs else None
        ws = pam.alloc_workspace(plan, F, x.shape[-1])
        pam.pam_fd_tea_tax(plan, x, img, nncc, pairs, ws)
        torch.cuda.synchronize()
        return img.cpu().numpy(), nncc.cpu().numpy(), None if pairs is None else pairs.cpu().numpy()
    finally:
        pam.pam_destroy(plan)


def check(img, rho, ref, tol_i=1e-5, tol_r=1e-4):
    e_i = float(np.linalg.norm(img - ref["I"]) / np.linalg.norm(ref["I"]))
    e_r = float(np.abs(rho - ref["rho_n"]).max())
    print(f"relL2(I)={e_i:.3e} max|d rho_n|={e_r:.3e}", flush=True)
    assert e_i <= tol_i and e_r <= tol_r


@pytest.mark.parametrize("n_sub", [3, 2, 1])
def test_fd_tea_small_workload(env, n_sub):
    g = synth.cfg1_geometry().replace(depths_m=(24.0 + 0.2 * np.arange(45)) * MM, n_sub=n_sub)
    rf = synth.batch(synth.cfg1_frame, [30, 31])
    img, rho, pairs = gpu_fd_tea(env, g, rf)
    for f in range(2):
        ref = T.fd_tea_tax(rf[f], g)
        check(img[f], rho[f], ref)
        if n_sub > 1:
            np.testing.assert_allclose(pairs[f], ref["rho"], atol=1e-4)
    # the focus sits at the emitter (0, 30 mm)
    d, j = np.unravel_index(np.argmax(img[0]), img[0].shape)
    assert abs(g.depths_m[d] - 30 * MM) <= 1 * MM


def test_fd_tea_benchmark_geometry_rows(env):
    """The 128-element, 4096-sample, 768-bin workload on 12 sampled depths (all 256 columns)."""
    g = synth.cfg2_geometry()
    g = g.replace(depths_m=g.depths_m[np.linspace(0, 511, 12).astype(int)])
    rf, _ = synth.cfg2_frame(7)
    img, rho, _ = gpu_fd_tea(env, g, rf[None])
    check(img[0], rho[0], T.fd_tea_tax(rf, g))


def test_fd_tea_stuff_lateral_and_degenerate_masks(env):
    """Zero-stuffed grid (pixels between elements) and a dead third sub-aperture."""
    g = synth.Geometry(n_elements=32, pitch_m=0.178 * MM, fs_hz=35.6e6, c_mps=1500.0, n_samples=512,
                       bands_hz=[(3e6, 15e6)], depths_m=(10 + 0.2 * np.arange(21)) * MM, n_x=64,
                       lateral="stuff", pattern_m=4)
    rng = np.random.default_rng(9)
    rf = synth.render(g, [synth.Emitter(0.5 * MM, 12 * MM, "broadband")], rng, snr_db=20.0)
    img, rho, _ = gpu_fd_tea(env, g, rf[None])
    check(img[0], rho[0], T.fd_tea_tax(rf, g))
    ones, zeros = np.ones(32, np.uint8), np.zeros(32, np.uint8)
    gd = g.replace(apod=np.stack([ones, ones, zeros]))
    img, rho, pairs = gpu_fd_tea(env, gd, rf[None])
    ref = T.fd_tea_tax(rf, gd)
    check(img[0], rho[0], ref)
    np.testing.assert_array_equal(pairs[0][1:], 0.0)
