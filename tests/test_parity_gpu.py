"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Stage checks read the stage results out of the workspace at the offsets the
library reports (pam_workspace_layout), so they see the same kernels as the
end-to-end call.  Tolerances for the FP32 path: relative L2 error of the image
<= 1e-5 and absolute NNCC error <= 1e-4 against the FP64 oracle.
"""
import numpy as np
import pytest

from oracle import as_tax as O
from paper_2412_02413_amd import synth

pytestmark = pytest.mark.gpu
MM = 1e-3
TOL_I = 1e-5
TOL_RHO = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def pam(torch_cuda):
    from paper_2412_02413_amd import pam as P
    P._lib()  # fails loudly if the library is missing
    return P


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def run(pam, torch, geom, rf, precision="fp32", want_pairs=True):
    plan = pam.pam_plan(geom, 0, precision)
    try:
        x = torch.from_numpy(np.ascontiguousarray(rf, dtype=np.float32)).cuda()
        out = pam.reconstruct(plan, x, want_nncc=True, want_pairs=want_pairs)
        torch.cuda.synchronize()
        lay = pam.pam_workspace_layout(plan, x.shape[0], x.shape[-1])
        res = {k: (v.cpu().numpy() if v is not None and k != "workspace" else v) for k, v in out.items()}
        res["layout"] = lay
        res["ws"] = out["workspace"]
        res["bins"] = pam.pam_plan_get_bins(plan)
        return res
    finally:
        pam.pam_destroy(plan)


def ws_view(torch, ws, offset, count, dtype):
    t = ws[offset: offset + count * np.dtype(dtype).itemsize]
    return t.cpu().numpy().view(dtype)


def check_end_to_end(res, ref, f=0, tol_i=TOL_I, tol_rho=TOL_RHO):
    e_i = rel_l2(res["image"][f], ref["I"])
    e_rho = float(np.abs(res["nncc"][f] - ref["rho_n"]).max())
    print(f"relL2(I)={e_i:.3e} max|d rho_n|={e_rho:.3e}", flush=True)
    assert e_i <= tol_i
    assert e_rho <= tol_rho


# ------------------------------------------------------------------ stages

def test_stage_time_fft_cfg1(pam, torch_cuda):
    g = synth.cfg1_geometry()
    rf = synth.batch(synth.cfg1_frame, [1, 2])
    res = run(pam, torch_cuda, g, rf)
    lay = res["layout"]
    F, n_sel, L = 2, lay.n_sel, g.n_elements
    X = ws_view(torch_cuda, res["ws"], lay.spectra, F * n_sel * L, np.complex64).reshape(F, n_sel, L)
    for f in range(F):
        ref = O.stage_outputs(rf[f], g)
        np.testing.assert_array_equal(res["bins"], ref["ks"])
        err = np.abs(X[f].T - ref["X"]).max() / np.abs(ref["X"]).max()
        assert err < 2e-6, err


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_stage_lateral_and_accumulators_cfg1(pam, torch_cuda, precision):
    """K2's coefficients and K3's accumulators on the 64-element workload (128 columns): in
    FP32 the coefficients are in the factored order of the vector-FFT fields kernel, in the
    split form in the folded order of the DFT-GEMM kernels."""
    g = synth.cfg1_geometry()
    rf = synth.batch(synth.cfg1_frame, [3])
    res = run(pam, torch_cuda, g, rf, precision=precision)
    lay = res["layout"]
    n_sel, N, ns = lay.n_sel, g.n_x, g.n_sub
    G = ws_view(torch_cuda, res["ws"], lay.coeffs, n_sel * ns * N, np.complex64).reshape(n_sel, ns, N)
    inv = ws_view(torch_cuda, res["ws"], lay.scales, n_sel, np.float32)
    ref = O.stage_outputs(rf[0], g)
    P = ref["P"]                                            # [n_sub][n_b][N]
    if precision == "fp32":
        # factored order: slot 16 r + q1 holds P((N/16) q1 + r) / N
        s = np.arange(N)
        want = P[:, :, (N // 16) * (s % 16) + s // 16] / N
    else:
        # folded coefficients: slot 2q = (P(q) + P(N-q))/N, slot 2q+1 = i (P(q) - P(N-q))/N,
        # ends P(0)/N and P(N/2)/N
        q = np.arange(1, N // 2)
        want = np.zeros((ns, n_sel, N), complex)
        want[:, :, 0] = P[:, :, 0] / N
        want[:, :, 1] = P[:, :, N // 2] / N
        want[:, :, 2 * q] = (P[:, :, q] + P[:, :, N - q]) / N
        want[:, :, 2 * q + 1] = 1j * (P[:, :, q] - P[:, :, N - q]) / N
    got = G.transpose(1, 0, 2) * inv[None, :, None]
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err < 2e-6, err
    # accumulators S_i, C_ij summed over the bin splits
    pix = g.n_z * N
    acc = ws_view(torch_cuda, res["ws"], lay.accum, lay.n_split * lay.n_acc * pix, np.float32)
    acc = acc.reshape(lay.n_split, 1, lay.n_acc, g.n_z, N).sum(axis=0)[0].astype(np.float64)
    cs = O.cross_spectra(rf[0], g)
    tol = 1e-5 if precision == "fp32" else 1e-4
    for i in range(3):
        assert rel_l2(acc[i], cs["S"][i]) < tol
    scale = np.sqrt(cs["S"][0] * cs["S"][1]).max()
    for c in range(3):
        assert np.abs(acc[3 + c] - cs["C"][c]).max() / scale < tol


# ------------------------------------------------------------------ end to end

@pytest.fixture(scope="module")
def cfg1_batch():
    return synth.batch(synth.cfg1_frame, [10, 11, 12])


def test_end_to_end_cfg1_batch(pam, torch_cuda, cfg1_batch):
    g = synth.cfg1_geometry()
    res = run(pam, torch_cuda, g, cfg1_batch)
    for f in range(cfg1_batch.shape[0]):
        ref = O.as_tax(cfg1_batch[f], g)
        check_end_to_end(res, ref, f)
        np.testing.assert_allclose(res["rho_pairs"][f], ref["rho"], atol=TOL_RHO)
        # the peak sits at the emitter (0, 30 mm)
        d, j = np.unravel_index(np.argmax(res["image"][f]), ref["I"].shape)
        assert abs(g.depths_m[d] - 30 * MM) <= 1 * MM


def test_batch_invariance_and_determinism(pam, torch_cuda, cfg1_batch):
    g = synth.cfg1_geometry()
    alone = run(pam, torch_cuda, g, cfg1_batch[1:2])
    mixed = run(pam, torch_cuda, g, cfg1_batch)
    again = run(pam, torch_cuda, g, cfg1_batch)
    np.testing.assert_array_equal(mixed["image"], again["image"])
    assert rel_l2(alone["image"][0], mixed["image"][1]) < 1e-6
    assert np.abs(alone["nncc"][0] - mixed["nncc"][1]).max() < 1e-5


def test_cfg2_reduced_depths(pam, torch_cuda):
    # cfg2 array, record length, bins and lateral grid; 70 depths (three tiles, ragged tail)
    g = synth.cfg2_geometry()
    g = g.replace(depths_m=g.depths_m[np.linspace(0, 511, 70).astype(int)])
    rf, _ = synth.cfg2_frame(5)
    res = run(pam, torch_cuda, g, rf[None])
    check_end_to_end(res, O.as_tax(rf, g))


def test_cfg2_full_size_sampled_rows(pam, torch_cuda):
    """Full cfg2 size (512 depths, 256 columns, 768 bins) in the benchmark's launch
    shape (64 frames); the oracle recomputes sampled depth rows of two frames."""
    g = synth.cfg2_geometry()
    frames = [synth.cfg2_frame(100 + s)[0] for s in range(4)]
    rf = np.stack([frames[i % 4] for i in range(64)])
    res = run(pam, torch_cuda, g, rf, want_pairs=False)
    lay = res["layout"]
    pix = g.n_z * g.n_x
    W = ws_view(torch_cuda, res["ws"], lay.weight, 64 * pix, np.float32).reshape(64, g.n_z, g.n_x)
    for f in (0, 37):
        rows = sorted({0, 255, 511, int(np.argmax(W[f].max(axis=1)))})
        gs = g.replace(depths_m=g.depths_m[rows])
        ref = O.as_tax(rf[f], gs)
        # weight and energy rows; the NNCC uses the GPU frame max, checked against the oracle there
        E = ws_view(torch_cuda, res["ws"], lay.energy, 64 * pix, np.float32).reshape(64, g.n_z, g.n_x)
        assert rel_l2(E[f][rows], ref["E"]) < 1e-5
        assert np.abs(W[f][rows] - ref["w"]).max() < 1e-4
        wmax = W[f].max()
        assert abs(wmax - ref["w"].max()) < 1e-4
        img = ref["w"] ** 2 / wmax ** 2 * ref["E"]
        assert rel_l2(res["image"][f][rows], img) < 1e-5
        np.testing.assert_allclose(res["image"][f], res["image"][f % 4], rtol=0, atol=0)


@pytest.mark.parametrize("n_sub", [1, 2])
def test_as_and_dax_variants(pam, torch_cuda, cfg1_batch, n_sub):
    g = synth.cfg1_geometry().replace(n_sub=n_sub)
    res = run(pam, torch_cuda, g, cfg1_batch[:1], want_pairs=n_sub > 1)
    ref = O.as_tax(cfg1_batch[0], g)
    check_end_to_end(res, ref)


def test_stuff_lateral_mode(pam, torch_cuda):
    # paper-style 2x zero-stuffing on a small array
    g = synth.Geometry(n_elements=32, pitch_m=0.178 * MM, fs_hz=35.6e6, c_mps=1500.0, n_samples=512,
                       bands_hz=[(3e6, 15e6)], depths_m=(10 + 0.2 * np.arange(45)) * MM, n_x=64,
                       lateral="stuff", pattern_m=4)
    rng = np.random.default_rng(9)
    em = [synth.Emitter(0.5 * MM, 14 * MM, "broadband")]
    rf = synth.render(g, em, rng, snr_db=20.0)
    res = run(pam, torch_cuda, g, rf[None])
    check_end_to_end(res, O.as_tax(rf, g))


def test_zero_evanescent_mode(pam, torch_cuda, cfg1_batch):
    g = synth.cfg1_geometry().replace(evanescent="zero", depths_m=(20 + 0.5 * np.arange(40)) * MM)
    res = run(pam, torch_cuda, g, cfg1_batch[:1])
    check_end_to_end(res, O.as_tax(cfg1_batch[0], g))


def test_shorter_records_on_a_long_plan(pam, torch_cuda):
    # plan for 8192 samples; 2048- and 4096-sample records use every 4th / 2nd plan bin
    g = synth.cfg3_geometry().replace(depths_m=(20 + 0.5 * np.arange(33)) * MM)
    for n_t in (2048, 4096):
        rng = np.random.default_rng(n_t)
        em = [synth.Emitter(1 * MM, 30 * MM, "broadband")]
        rf = synth.render(g, em, rng, n_t=n_t)
        res = run(pam, torch_cuda, g, rf[None])
        check_end_to_end(res, O.as_tax(rf, g.replace(n_samples=n_t)))


def test_zero_frames_is_a_no_op(pam, torch_cuda):
    torch = torch_cuda
    plan = pam.pam_plan(synth.cfg1_geometry(), 0)
    try:
        rf = torch.empty((0, 64, 1024), device="cuda")
        img = torch.empty((0, 151, 128), device="cuda")
        pam.pam_as_tax(plan, rf, img, workspace=None)
    finally:
        pam.pam_destroy(plan)


def test_workspace_too_small_is_rejected(pam, torch_cuda):
    torch = torch_cuda
    plan = pam.pam_plan(synth.cfg1_geometry(), 0)
    try:
        rf = torch.zeros((1, 64, 1024), device="cuda")
        img = torch.full((1, 151, 128), -7.0, device="cuda")
        ws = torch.empty(pam.pam_workspace_size(plan, 1) - 256, dtype=torch.uint8, device="cuda")
        with pytest.raises(pam.PamError) as ei:
            pam.pam_as_tax(plan, rf, img, workspace=ws)
        assert ei.value.status == pam.PAM_ERR_WORKSPACE
        torch.cuda.synchronize()
        assert bool((img == -7.0).all())    # nothing written
    finally:
        pam.pam_destroy(plan)


# ------------------------------------------------------------------ lateral grid sizes
# The fields kernel has three tilings selected by the lateral size N: the factored
# two-stage transform (N = 256: 16 depths per workgroup; N = 512: 8 depths, even and odd
# wavenumbers combined), 16 depths x 64 CT columns (other multiples of 64), 32 depths x
# 32 NW columns (the remaining multiples of 32).  Each grid below reaches one of them
# with a ragged depth tail; the split form runs too.
SPLIT_TOL = (1e-3, 1e-3)


def _grid_case(n_elements, n_x, n_depths, seed):
    g = synth.Geometry(n_elements=n_elements, pitch_m=0.3 * MM, fs_hz=20e6, c_mps=1540.0, n_samples=256,
                       bands_hz=[(2e6, 6e6)], depths_m=(15 + 0.4 * np.arange(n_depths)) * MM, n_x=n_x,
                       lateral="pad")
    rng = np.random.default_rng(seed)
    em = [synth.Emitter(-1.0 * MM, 19 * MM, "broadband"), synth.Emitter(2.0 * MM, 24 * MM, "broadband")]
    return g, synth.render(g, em, rng, snr_db=20.0)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("n_elements,n_x,n_depths", [(64, 512, 45), (32, 96, 37), (48, 192, 21)])
def test_lateral_grid_sizes(pam, torch_cuda, precision, n_elements, n_x, n_depths):
    g, rf = _grid_case(n_elements, n_x, n_depths, seed=n_x)
    res = run(pam, torch_cuda, g, rf[None], precision=precision)
    tol_i, tol_rho = (TOL_I, TOL_RHO) if precision == "fp32" else SPLIT_TOL
    check_end_to_end(res, O.as_tax(rf, g), tol_i=tol_i, tol_rho=tol_rho)


def test_band_union(pam, torch_cuda, cfg1_batch):
    """Omega as a union of two disjoint windows (frequency-selective map)."""
    g = synth.cfg1_geometry().replace(bands_hz=[(1.2e6, 1.8e6), (2.8e6, 3.4e6)],
                                      depths_m=(20 + 0.5 * np.arange(45)) * MM)
    res = run(pam, torch_cuda, g, cfg1_batch[:1])
    assert len(res["bins"]) == len(O.bins(g.fs_hz, g.n_samples, g.bands_hz))
    check_end_to_end(res, O.as_tax(cfg1_batch[0], g))


@pytest.mark.parametrize("case", ["dead_third", "identical"])
def test_degenerate_masks(pam, torch_cuda, case):
    """Degenerate apodization sets against the oracle.  dead_third: a_3 is empty, so S_3 = 0
    and the two pairs that hold it have a zero denominator (0, then the eps floor); the
    weight is eps^(2/3) everywhere.  identical: a_1 = a_2 = a_3, so every pair reaches the
    upper clamp and rho_n = 1."""
    g = synth.cfg1_geometry().replace(depths_m=(24.0 + 0.2 * np.arange(37)) * MM)
    rf = synth.batch(synth.cfg1_frame, [16])
    ones, zeros = np.ones(64, np.uint8), np.zeros(64, np.uint8)
    apod = np.stack([ones, ones, zeros]) if case == "dead_third" else np.stack([ones, ones, ones])
    gg = g.replace(apod=apod)
    res = run(pam, torch_cuda, gg, rf)
    ref = O.as_tax(rf[0], gg)
    check_end_to_end(res, ref)
    np.testing.assert_allclose(res["rho_pairs"][0], ref["rho"], atol=TOL_RHO)
    np.testing.assert_allclose(res["nncc"][0], 1.0, atol=TOL_RHO)
    if case == "dead_third":
        np.testing.assert_array_equal(res["rho_pairs"][0][1:], 0.0)


def test_binding_rejects_misshaped_buffers(pam, torch_cuda):
    """The binding checks device, dtype, contiguity and shape against the plan before any
    launch: a wrong channel count or a short image is rejected and nothing is written."""
    torch = torch_cuda
    g = synth.cfg1_geometry()
    plan = pam.pam_plan(g, 0)
    try:
        ws = pam.alloc_workspace(plan, 1)
        img = torch.full((1, g.n_z, g.n_x), -7.0, device="cuda")
        with pytest.raises(pam.PamError):
            pam.pam_as_tax(plan, torch.zeros((1, 63, 1024), device="cuda"), img, workspace=ws)
        with pytest.raises(pam.PamError):
            pam.pam_as_tax(plan, torch.zeros((1, 64, 1024), device="cuda"), img[:, :-1], workspace=ws)
        with pytest.raises(pam.PamError):
            pam.pam_as_tax(plan, torch.zeros((1, 64, 1024), device="cuda", dtype=torch.float64), img,
                           workspace=ws)
        torch.cuda.synchronize()
        assert bool((img == -7.0).all())
    finally:
        pam.pam_destroy(plan)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16", "split_fp16", "bf16"])
@pytest.mark.parametrize("n_sub", [1, 2, 3])
def test_factored_transform_forms(pam, torch_cuda, precision, n_sub):
    """N = 256 (the factored two-stage transform) in every sub-aperture count and operand form,
    two frames, 37 depths (three 16-depth tiles, ragged tail)."""
    g = synth.cfg2_geometry()
    g = g.replace(depths_m=g.depths_m[np.linspace(0, 511, 37).astype(int)], n_sub=n_sub)
    rf = np.stack([synth.cfg2_frame(300 + s)[0] for s in range(2)])
    res = run(pam, torch_cuda, g, rf, precision=precision, want_pairs=n_sub > 1)
    tol_i, tol_rho = {"fp32": (TOL_I, TOL_RHO), "bf16": (1e-2, 5e-2)}.get(precision, SPLIT_TOL)
    for f in range(2):
        check_end_to_end(res, O.as_tax(rf[f], g), f, tol_i=tol_i, tol_rho=tol_rho)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16", "split_fp16"])
def test_largest_serving_frame(pam, torch_cuda, precision):
    """The largest serving frame's array and record: 256 elements at 0.2 mm on 512 columns,
    16384 samples at 20 MHz.  A 159-bin band (2.0-2.195 MHz) and 32 depths keep the oracle
    affordable while the path still runs the 8192-point time FFT, the 256-element lateral
    DFT and the 512-column fields kernel."""
    g = synth.cfg5_geometry(256, 20e6, 16384)
    df = g.fs_hz / g.n_samples
    g = g.replace(bands_hz=[(2.0e6, 2.0e6 + 159.5 * df)],
                  depths_m=g.depths_m[np.linspace(0, len(g.depths_m) - 1, 32).astype(int)])
    rng = np.random.default_rng(77)
    em = [synth.Emitter(-3 * MM, 30 * MM, "broadband"), synth.Emitter(4 * MM, 45 * MM, "broadband")]
    rf = synth.render(g, em, rng, snr_db=20.0)
    res = run(pam, torch_cuda, g, rf[None], precision=precision)
    ref = O.as_tax(rf, g)
    assert len(res["bins"]) == len(O.bins(g.fs_hz, g.n_samples, g.bands_hz)) == 159
    tol_i, tol_rho = (TOL_I, TOL_RHO) if precision == "fp32" else SPLIT_TOL
    check_end_to_end(res, ref, tol_i=tol_i, tol_rho=tol_rho)


def test_graph_replay_matches_eager(pam, torch_cuda):
    """pam_as_tax captured once into a HIP graph (its launches only: the call allocates and
    clears nothing) and replayed four times, each time on new frames copied into the captured
    input, with eager work and synchronisations between the replays: every replay equals the
    eager call on the same frames bit for bit."""
    torch = torch_cuda
    g = synth.cfg1_geometry()
    frames = synth.batch(synth.cfg1_frame, [11, 12, 13, 14, 15, 16, 17, 18])
    plan = pam.pam_plan(g, 0, "fp32")
    try:
        x = torch.from_numpy(frames[:2]).cuda()
        img, nn = torch.empty((2, g.n_z, g.n_x), device="cuda"), torch.empty((2, g.n_z, g.n_x), device="cuda")
        ws = pam.alloc_workspace(plan, 2, g.n_samples)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            pam.pam_as_tax(plan, x, img, nn, None, ws, s)
        s.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            pam.pam_as_tax(plan, x, img, nn, None, ws, s)
        torch.cuda.synchronize()
        for k in range(4):
            x.copy_(torch.from_numpy(frames[2 * k:2 * k + 2]))
            img.zero_()
            nn.zero_()
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            got_i, got_n = img.clone(), nn.clone()
            # the eager call on the same frames, with its own buffers
            img_e, nn_e = torch.empty_like(img), torch.empty_like(nn)
            pam.pam_as_tax(plan, x, img_e, nn_e, None, pam.alloc_workspace(plan, 2, g.n_samples))
            torch.cuda.synchronize()
            assert torch.equal(got_i, img_e) and torch.equal(got_n, nn_e), k
        del graph
    finally:
        pam.pam_destroy(plan)


@pytest.mark.parametrize("n_t,L", [(32, 8), (256, 8), (256, 7), (2048, 6), (4096, 8), (4096, 9), (16384, 8)])
def test_stage_time_fft_record_lengths(pam, torch_cuda, n_t, L):
    """K1 (the time FFT) on every pass structure it runs: 32 samples (radix 8 then 2),
    256 (8, 8, 2), 2048 (8, 8, 8, 2), 4096 (8, 8, 8, 4), 16384 (8, 8, 8, 8, 2 with 32 points
    per thread); two channels per workgroup where 2 divides L (up to 4096 samples), one
    otherwise (L = 7 and 9, and 16384 samples)."""
    g = synth.Geometry(n_elements=L, pitch_m=0.3 * MM, fs_hz=20e6, c_mps=1540.0, n_samples=n_t,
                       bands_hz=[(0.0, 10e6)], depths_m=np.array([20.0, 20.5]) * MM, n_x=32, lateral="pad")
    rng = np.random.default_rng(n_t + L)
    rf = rng.standard_normal((2, L, n_t)).astype(np.float32)
    res = run(pam, torch_cuda, g, rf)
    lay = res["layout"]
    F, n_sel = 2, lay.n_sel
    assert n_sel == n_t // 2 - 1
    X = ws_view(torch_cuda, res["ws"], lay.spectra, F * n_sel * L, np.complex64).reshape(F, n_sel, L)
    for f in range(F):
        ref = O.stage_outputs(rf[f], g)
        err = np.abs(X[f].T - ref["X"]).max() / np.abs(ref["X"]).max()
        print(f"n_t={n_t}: max |dX| / max |X| = {err:.2e}", flush=True)
        assert err < 2e-6, err


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_coherence_pair_sums(pam, torch_cuda, precision):
    """Adjacent-pixel cross-spectra (the coherence channels of an n_sub = 1 plan) against the
    oracle's pair sums: 38 depths (three 16-depth tiles, ragged tail), full-size lateral grid,
    two frames.  The image of such a plan stays the plain AS image."""
    g = synth.cfg2_geometry()
    g = g.replace(depths_m=g.depths_m[np.linspace(0, 511, 38).astype(int)], n_sub=1,
                  apod=np.ones((1, g.n_elements), np.uint8), coherence=1)
    rf = np.stack([synth.cfg2_frame(310 + s)[0] for s in range(2)])
    res = run(pam, torch_cuda, g, rf, precision=precision, want_pairs=False)
    lay = res["layout"]
    assert lay.n_acc == 5
    nz, nx = len(g.depths_m), g.n_x
    acc = ws_view(torch_cuda, res["ws"], lay.accum, lay.n_split * 2 * 5 * nz * nx, np.float32)
    acc = acc.reshape(lay.n_split, 2, 5, nz, nx).astype(np.float64).sum(axis=0)
    tol = 2e-5 if precision == "fp32" else 2e-4
    for f in range(2):
        ref = O.pair_cross_spectra(rf[f], g)
        smax = ref["S"].max()
        gx = acc[f, 1] + 1j * acc[f, 2]
        gz = acc[f, 3] + 1j * acc[f, 4]
        e = [float(np.abs(acc[f, 0] - ref["S"]).max() / smax),
             float(np.abs(gx - ref["Gx"]).max() / smax),
             float(np.abs(gz - ref["Gz"]).max() / smax)]
        print(f"frame {f}: max err / max S  S={e[0]:.2e} Gx={e[1]:.2e} Gz={e[2]:.2e}", flush=True)
        assert max(e) <= tol
        # normalised coherence where the field is not negligible
        x1, z1 = np.arange(nx) ^ 1, np.arange(nz) ^ 1
        live = (ref["S"] > 1e-2 * smax) & (ref["S"][:, x1] > 1e-2 * smax) & (ref["S"][z1, :] > 1e-2 * smax)
        cx = np.abs(gx) / np.sqrt(acc[f, 0] * acc[f, 0][:, x1])
        cx_ref = np.abs(ref["Gx"]) / np.sqrt(ref["S"] * ref["S"][:, x1])
        assert np.abs(cx - cx_ref)[live].max() <= 100 * tol
        check_end_to_end(res, O.as_tax(rf[f], g), f, *((TOL_I, TOL_RHO) if precision == "fp32" else SPLIT_TOL))


def test_coherence_needs_one_subaperture(pam, torch_cuda):
    g = synth.cfg2_geometry().replace(coherence=1)
    with pytest.raises(pam.PamError):
        pam.pam_plan(g, 0, "fp32")
    g = synth.cfg2_geometry()
    g = g.replace(depths_m=g.depths_m[:37], n_sub=1, apod=np.ones((1, g.n_elements), np.uint8), coherence=1)
    with pytest.raises(pam.PamError):
        pam.pam_plan(g, 0, "fp32")


@pytest.mark.parametrize("precision", ["fp32", "split_bf16", "split_fp16", "bf16"])
@pytest.mark.parametrize("n_sub", [1, 2, 3])
def test_factored_512_forms(pam, torch_cuda, precision, n_sub):
    """N = 512 on the factored kernel (two 256-point transforms over even and odd
    wavenumbers, combined per pixel pair x, x + 256) in every sub-aperture count and operand
    form: 13 depths (one full 8-depth tile and a ragged one), two frames."""
    g, rf0 = _grid_case(64, 512, 13, seed=5120)
    g = g.replace(n_sub=n_sub)
    _, rf1 = _grid_case(64, 512, 13, seed=5121)
    rf = np.stack([rf0, rf1])
    res = run(pam, torch_cuda, g, rf, precision=precision, want_pairs=n_sub > 1)
    tol_i, tol_rho = {"fp32": (TOL_I, TOL_RHO), "bf16": (1e-2, 5e-2)}.get(precision, SPLIT_TOL)
    for f in range(2):
        check_end_to_end(res, O.as_tax(rf[f], g), f, tol_i=tol_i, tol_rho=tol_rho)


def test_injected_allocation_failure_leaks_nothing(pam, torch_cuda):
    """An out-of-memory at any point of plan building returns PAM_ERR_OOM and releases every
    table the plan had allocated (checked by the library's live-allocation count)."""
    g = synth.cfg1_geometry()
    base = pam.debug_live_allocations()
    plan = pam.pam_plan(g, 0, "fp32")
    n_allocs = pam.debug_live_allocations() - base
    pam.pam_destroy(plan)
    assert n_allocs > 5 and pam.debug_live_allocations() == base
    try:
        for k in sorted({0, 1, 2, n_allocs // 2, n_allocs - 1}):
            pam.debug_fail_allocation(k)
            with pytest.raises(pam.PamError) as err:
                pam.pam_plan(g, 0, "fp32")
            assert err.value.status == -2           # PAM_ERR_OOM
            assert pam.debug_live_allocations() == base
        # past the last allocation the injection never fires: the plan builds and still works
        pam.debug_fail_allocation(n_allocs + 5)
        plan = pam.pam_plan(g, 0, "fp32")
    finally:
        pam.debug_fail_allocation(-1)
    try:
        rf = synth.cfg1_frame(9)
        res = pam.reconstruct(plan, torch_cuda.from_numpy(rf[None]).cuda())
        torch_cuda.cuda.synchronize()
        assert np.isfinite(res["image"].cpu().numpy()).all()
    finally:
        pam.pam_destroy(plan)
    assert pam.debug_live_allocations() == base


@pytest.mark.parametrize("geom_name", ["cfg1", "cfg2", "cfg3"])
def test_workspace_never_shrinks(pam, torch_cuda, geom_name):
    """The bin split changes with the frame count, but the workspace size never shrinks
    as frames or record length grow, and the accum region always holds the n_split F
    planes the chosen split writes; a workspace sized for 64 frames then serves a call of
    23 frames with the same results as a workspace sized for 23."""
    g = getattr(synth, f"{geom_name}_geometry")()
    plan = pam.pam_plan(g, 0, "fp32")
    try:
        pix = g.n_z * g.n_x
        lengths = [g.n_samples >> j for j in range(3)][::-1]
        prev_t = 0
        for n_t in lengths:
            prev = 0
            for F in list(range(0, 70)) + [96, 128, 200]:
                lay = pam.pam_workspace_layout(plan, F, n_t)
                assert lay.total >= prev, (n_t, F)
                prev = lay.total
                room = (lay.energy - lay.accum) // 4
                assert room >= lay.n_split * F * lay.n_acc * pix, (n_t, F, lay.n_split)
            assert pam.pam_workspace_size(plan, 64, n_t) >= prev_t
            prev_t = pam.pam_workspace_size(plan, 64, n_t)
        F = 23
        rf = np.stack([synth.cfg1_frame(s) for s in range(F)]) if geom_name == "cfg1" else None
        if rf is not None:
            x = torch_cuda.from_numpy(rf).cuda()
            outs = []
            for n_ws in (F, 64):
                ws = pam.alloc_workspace(plan, n_ws, g.n_samples)
                img = torch_cuda.empty((F, g.n_z, g.n_x), device="cuda")
                pam.pam_as_tax(plan, x, img, None, None, ws)
                torch_cuda.cuda.synchronize()
                outs.append(img.cpu().numpy())
            np.testing.assert_array_equal(outs[0], outs[1])
    finally:
        pam.pam_destroy(plan)
