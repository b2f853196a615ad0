"""C-ABI checks that need no GPU: exported symbols, argument validation and
error codes (every validation error is returned before any device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2412_02413_amd import pam as P
from paper_2412_02413_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*(pam_[a-z_]+)\s*\(", txt, flags=re.M))
    return sorted(names)


def test_library_exports_every_declared_function():
    lib = P._lib()
    names = header_functions()
    assert {"pam_plan", "pam_as_tax", "pam_destroy", "pam_workspace_size"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def plan_status(geom, precision="fp32"):
    g, keep = P.geometry_struct(geom, precision)
    h = C.c_void_p(12345)
    st = P._lib().pam_plan(C.byref(g), 0, C.byref(h))
    if st == 0:
        P._lib().pam_destroy(h)
    else:
        assert h.value is None      # *out is NULL on failure
    return st


@pytest.mark.parametrize("change,status", [
    (dict(n_x=48), P.PAM_ERR_INVALID_ARG),                # N_x < L
    (dict(n_x=144), P.PAM_ERR_UNSUPPORTED),               # not a multiple of 32
    (dict(n_samples=1000), P.PAM_ERR_UNSUPPORTED),        # not a power of two
    (dict(n_x=1024), P.PAM_ERR_UNSUPPORTED),              # wider than the kernels' LDS tiles
    (dict(n_samples=32768), P.PAM_ERR_UNSUPPORTED),       # beyond the LDS FFT
    (dict(bands_hz=[(6e6, 5e6)]), P.PAM_ERR_INVALID_ARG), # lo > hi
    (dict(bands_hz=[(9.99e6, 9.999e6)]), P.PAM_ERR_INVALID_ARG),  # no bin in band
    (dict(pitch_m=float("nan")), P.PAM_ERR_INVALID_ARG),
    (dict(c_mps=0.0), P.PAM_ERR_INVALID_ARG),
    (dict(depths_m=np.array([0.02, -0.001])), P.PAM_ERR_INVALID_ARG),
    (dict(depths_m=np.array([0.02, float("inf")])), P.PAM_ERR_INVALID_ARG),
    (dict(n_sub=4), P.PAM_ERR_INVALID_ARG),
    (dict(lateral="stuff", n_x=96), P.PAM_ERR_INVALID_ARG),      # 96 / 64 not an integer
    (dict(eps=1.5), P.PAM_ERR_INVALID_ARG),
])
def test_plan_rejects_invalid_geometry(change, status):
    g = synth.cfg1_geometry().replace(**change)
    assert plan_status(g) == status


def test_plan_rejects_non_binary_mask():
    a = np.ones((3, 64), np.uint8)
    a[1, 5] = 2
    assert plan_status(synth.cfg1_geometry().replace(apod=a)) == P.PAM_ERR_INVALID_ARG


def test_null_arguments():
    lib = P._lib()
    assert lib.pam_plan(None, 0, None) == P.PAM_ERR_INVALID_ARG
    assert lib.pam_as_tax(None, None, 1, 1024, None, None, None, None, 0, None) == P.PAM_ERR_INVALID_ARG
    n = C.c_size_t()
    assert lib.pam_workspace_size(None, 1, 1024, C.byref(n)) == P.PAM_ERR_INVALID_ARG
    lib.pam_destroy(None)          # NULL-safe
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.pam_status_string(s)


def test_valid_geometry_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert plan_status(synth.cfg1_geometry()) == P.PAM_ERR_DEVICE


def test_grouped_binding_checks_on_cpu():
    """pam_as_tax_grouped rejects, before any library call, an empty group list, a packed RF
    of the wrong size, a short image, a non-float32 buffer and (here) host tensors."""
    import torch
    info = P.PlanInfoC(n_bins=1639, n_z=151, n_x=128, n_sub=3, n_elements=64, n_samples=8192, n_pairs=3,
                       device=0)
    plan = P.Plan(0, None, "fp32", info)
    groups = [(2048, 2), (4096, 1)]
    rf = torch.zeros(64 * (2 * 2048 + 4096))
    img = torch.zeros((3, 151, 128))
    cases = [
        ([], rf, img),
        (groups, torch.zeros(64 * (2 * 2048 + 4096) - 1), img),
        (groups, rf, torch.zeros((2, 151, 128))),
        (groups, rf.double(), img),
        (groups, rf, img),                                   # right sizes, but not on the GPU
    ]
    for g, r, i in cases:
        with pytest.raises(P.PamError) as ei:
            P.pam_as_tax_grouped(plan, r, g, i)
        assert ei.value.status == P.PAM_ERR_INVALID_ARG


def test_binding_buffer_checks_on_cpu():
    """check_buffers rejects a wrong channel count, a short image, a non-float32 RF, a
    non-contiguous view and (here) host tensors, each before any library call."""
    import torch
    info = P.PlanInfoC(n_bins=205, n_z=151, n_x=128, n_sub=3, n_elements=64, n_samples=1024, n_pairs=3,
                       device=0)
    rf = torch.zeros((2, 64, 1024))
    img = torch.zeros((2, 151, 128))
    cases = [
        (torch.zeros((2, 63, 1024)), img, None),
        (rf, torch.zeros((2, 150, 128)), None),
        (rf.double(), img, None),
        (rf, torch.zeros((2, 128, 151)).transpose(1, 2), None),
        (rf, img, torch.zeros((2, 1, 151, 128))),
        (rf, img, None),                                   # right shapes, but not on the GPU
    ]
    for r, i, pairs in cases:
        with pytest.raises(P.PamError) as ei:
            P.check_buffers(info, r, i, None, pairs, None)
        assert ei.value.status == P.PAM_ERR_INVALID_ARG
