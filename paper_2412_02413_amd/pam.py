"""Thin ctypes binding of libpam (include/pam.h): argument marshalling only.

Every step of the reconstruction runs in the HIP library; PyTorch supplies
device memory and streams.  The library must be built (``build.py`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpam.so")

PAM_OK, PAM_ERR_INVALID_ARG, PAM_ERR_OOM, PAM_ERR_DEVICE, PAM_ERR_UNSUPPORTED, PAM_ERR_WORKSPACE = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp32": 0, "split_bf16": 1, "split_fp16": 2, "bf16": 3, "fp16": 4}
LATERAL = {"pad": 0, "stuff": 1}
EVANESCENT = {"decay": 0, "zero": 1}


class PamError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_lib().pam_status_string(status).decode()} ({status})")
        self.status = status


class GeometryC(C.Structure):
    _fields_ = [("n_elements", C.c_int32), ("pitch_m", C.c_double), ("fs_hz", C.c_double),
                ("c_mps", C.c_double), ("n_samples", C.c_int32), ("n_bands", C.c_int32),
                ("band_lo_hz", C.POINTER(C.c_double)), ("band_hi_hz", C.POINTER(C.c_double)),
                ("n_depths", C.c_int32), ("depths_m", C.POINTER(C.c_double)), ("n_x", C.c_int32),
                ("lateral", C.c_int), ("n_sub", C.c_int32), ("apod", C.POINTER(C.c_uint8)),
                ("pattern_m", C.c_int32), ("eps", C.c_double), ("precision", C.c_int),
                ("evanescent", C.c_int), ("coherence", C.c_int32)]


class PlanInfoC(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("n_z", C.c_int32), ("n_x", C.c_int32), ("n_sub", C.c_int32),
                ("n_elements", C.c_int32), ("n_samples", C.c_int32), ("n_pairs", C.c_int32),
                ("device", C.c_int32)]


class GroupC(C.Structure):
    _fields_ = [("n_t", C.c_int32), ("n_frames", C.c_int64)]


class LayoutC(C.Structure):
    _fields_ = [("spectra", C.c_size_t), ("coeffs", C.c_size_t), ("scales", C.c_size_t),
                ("accum", C.c_size_t), ("energy", C.c_size_t), ("weight", C.c_size_t),
                ("blockmax", C.c_size_t), ("total", C.c_size_t), ("n_sel", C.c_int32),
                ("n_split", C.c_int32), ("n_acc", C.c_int32)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        # torch first: its HIP runtime (same soname) is then the one libpam binds to,
        # so torch streams and device pointers are valid in the library.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run paper_2412_02413_amd/build.py or __graft_entry__.build())")
        lib = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        lib.pam_plan.argtypes = [C.POINTER(GeometryC), C.c_int, C.POINTER(vp)]
        lib.pam_plan.restype = C.c_int
        lib.pam_plan_get_info.argtypes = [vp, C.POINTER(PlanInfoC)]
        lib.pam_plan_get_info.restype = C.c_int
        lib.pam_plan_get_bins.argtypes = [vp, C.POINTER(i32), i32]
        lib.pam_plan_get_bins.restype = C.c_int
        lib.pam_workspace_size.argtypes = [vp, i64, i32, C.POINTER(sz)]
        lib.pam_workspace_size.restype = C.c_int
        lib.pam_workspace_layout.argtypes = [vp, i64, i32, C.POINTER(LayoutC)]
        lib.pam_workspace_layout.restype = C.c_int
        lib.pam_as_tax.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, sz, vp]
        lib.pam_as_tax.restype = C.c_int
        lib.pam_as_tax_events.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, sz, vp, C.POINTER(vp)]
        lib.pam_as_tax_events.restype = C.c_int
        lib.pam_fd_tea_tax.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, sz, vp]
        lib.pam_fd_tea_tax.restype = C.c_int
        lib.pam_as_tax_noalloc.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp]
        lib.pam_as_tax_noalloc.restype = C.c_int
        lib.pam_destroy.argtypes = [vp]
        lib.pam_destroy.restype = None
        lib.pam_status_string.argtypes = [C.c_int]
        lib.pam_status_string.restype = C.c_char_p
        lib.pam_workspace_size_grouped.argtypes = [vp, C.POINTER(GroupC), i32, C.POINTER(sz)]
        lib.pam_workspace_size_grouped.restype = C.c_int
        lib.pam_as_tax_grouped.argtypes = [vp, vp, C.POINTER(GroupC), i32, vp, vp, vp, vp, sz, vp]
        lib.pam_as_tax_grouped.restype = C.c_int
        lib.pam_debug_fail_allocation.argtypes = [i32]
        lib.pam_debug_fail_allocation.restype = None
        lib.pam_debug_grouped_one_launch.argtypes = [vp, vp, i32]
        lib.pam_debug_grouped_one_launch.restype = C.c_int32
        lib.pam_debug_live_allocations.argtypes = []
        lib.pam_debug_live_allocations.restype = i64
        _LIB = lib
    return _LIB


def _check(status: int, what: str):
    if status != PAM_OK:
        raise PamError(status, what)


def geometry_struct(geom, precision: Optional[str] = None):
    """Marshal a Geometry (synth.Geometry or anything with the same fields) into pam_geometry_t.

    Returns the struct and the numpy arrays it points into (keep them alive)."""
    lo = np.ascontiguousarray([b[0] for b in geom.bands_hz], dtype=np.float64)
    hi = np.ascontiguousarray([b[1] for b in geom.bands_hz], dtype=np.float64)
    z = np.ascontiguousarray(geom.depths_m, dtype=np.float64)
    keep = [lo, hi, z]
    g = GeometryC()
    g.n_elements = geom.n_elements
    g.pitch_m = geom.pitch_m
    g.fs_hz = geom.fs_hz
    g.c_mps = geom.c_mps
    g.n_samples = geom.n_samples
    g.n_bands = len(lo)
    g.band_lo_hz = lo.ctypes.data_as(C.POINTER(C.c_double))
    g.band_hi_hz = hi.ctypes.data_as(C.POINTER(C.c_double))
    g.n_depths = len(z)
    g.depths_m = z.ctypes.data_as(C.POINTER(C.c_double))
    g.n_x = geom.n_x
    g.lateral = LATERAL[geom.lateral]
    g.n_sub = geom.n_sub
    if getattr(geom, "apod", None) is not None:
        ap = np.ascontiguousarray(geom.apod, dtype=np.uint8)
        keep.append(ap)
        g.apod = ap.ctypes.data_as(C.POINTER(C.c_uint8))
    else:
        g.apod = None
    g.pattern_m = getattr(geom, "pattern_m", 16)
    g.eps = geom.eps
    g.precision = PRECISIONS[precision or getattr(geom, "precision", "fp32")]
    g.evanescent = EVANESCENT[geom.evanescent]
    g.coherence = int(getattr(geom, "coherence", 0))
    return g, keep


@dataclass
class Plan:
    handle: int
    geom: object
    precision: str
    info: PlanInfoC

    @property
    def n_z(self):
        return self.info.n_z

    @property
    def n_x(self):
        return self.info.n_x

    @property
    def n_pairs(self):
        return self.info.n_pairs


def pam_plan(geom, device: int = 0, precision: str = "fp32") -> Plan:
    g, keep = geometry_struct(geom, precision)
    h = C.c_void_p()
    _check(_lib().pam_plan(C.byref(g), device, C.byref(h)), "pam_plan")
    info = PlanInfoC()
    _check(_lib().pam_plan_get_info(h, C.byref(info)), "pam_plan_get_info")
    del keep
    return Plan(h.value, geom, precision, info)


def _groups(groups):
    """(n_t, n_frames) pairs -> a pam_group_t array."""
    arr = (GroupC * len(groups))()
    for k, (n_t, F) in enumerate(groups):
        arr[k].n_t, arr[k].n_frames = int(n_t), int(F)
    return arr


def pam_workspace_size_grouped(plan: Plan, groups) -> int:
    n = C.c_size_t(0)
    _check(_lib().pam_workspace_size_grouped(C.c_void_p(plan.handle), _groups(groups), len(groups), C.byref(n)),
           "pam_workspace_size_grouped")
    return n.value


def alloc_workspace_grouped(plan: Plan, groups, device="cuda"):
    import torch
    return torch.empty(pam_workspace_size_grouped(plan, groups), dtype=torch.uint8, device=device)


def pam_as_tax_grouped(plan: Plan, rf, groups, image, nncc=None, rho_pairs=None, workspace=None, stream=None):
    """Frames of several record lengths in one call: groups = [(n_t, n_frames), ...], rf a
    contiguous float32 device tensor holding the groups back to back ([n_frames][L][n_t] each),
    image / nncc [sum n_frames][n_z][n_x] (rho_pairs [..][n_pairs][n_z][n_x]) in that order."""
    import torch
    info = plan.info
    F = sum(int(f) for _, f in groups)
    want_rf = sum(int(f) * info.n_elements * int(n) for n, f in groups)

    def bad(msg):
        raise PamError(-1, f"pam_as_tax_grouped: {msg}")

    if not groups or any(int(f) < 0 for _, f in groups):
        bad("groups must be a non-empty list of (n_t, n_frames >= 0)")
    for name, t, count in (("rf", rf, want_rf), ("image", image, F * info.n_z * info.n_x),
                           ("nncc", nncc, F * info.n_z * info.n_x),
                           ("rho_pairs", rho_pairs, F * info.n_pairs * info.n_z * info.n_x)):
        if t is None:
            if name in ("rf", "image"):
                bad(f"{name} is required")
            continue
        if not (t.dtype == torch.float32 and t.is_contiguous()):
            bad(f"{name} must be a contiguous float32 tensor")
        if t.numel() != count:
            bad(f"{name} holds {t.numel()} values, expected {count}")
    for name, t in (("rf", rf), ("image", image), ("nncc", nncc), ("rho_pairs", rho_pairs),
                    ("workspace", workspace)):
        if t is not None and (t.device.type != "cuda" or t.device.index != info.device):
            bad(f"{name} must live on cuda:{info.device}, got {t.device}")
    stream = stream or torch.cuda.current_stream()
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(_lib().pam_as_tax_grouped(C.c_void_p(plan.handle), _ptr(rf), _groups(groups), len(groups), _ptr(image),
                                     _ptr(nncc), _ptr(rho_pairs), _ptr(workspace), ws_bytes,
                                     C.c_void_p(stream.cuda_stream)), "pam_as_tax_grouped")


def debug_fail_allocation(n: int) -> None:
    """Make the n-th next device allocation of plan building fail as out of memory (n < 0 disarms)."""
    _lib().pam_debug_fail_allocation(n)


def debug_live_allocations() -> int:
    """Device allocations held by all live plans of the process."""
    return int(_lib().pam_debug_live_allocations())


def debug_grouped_one_launch(plan: Plan, groups) -> bool:
    """Whether pam_as_tax_grouped with these (n_t, n_frames) groups runs its fields stage as
    one grouped launch (else one launch per group)."""
    r = int(_lib().pam_debug_grouped_one_launch(C.c_void_p(plan.handle), _groups(groups), len(groups)))
    _check(min(r, 0), "pam_debug_grouped_one_launch")
    return r == 1


def pam_destroy(plan: Plan) -> None:
    if plan is not None and plan.handle:
        _lib().pam_destroy(C.c_void_p(plan.handle))
        plan.handle = 0


def pam_plan_get_bins(plan: Plan) -> np.ndarray:
    out = np.zeros(plan.info.n_bins, dtype=np.int32)
    _check(_lib().pam_plan_get_bins(C.c_void_p(plan.handle), out.ctypes.data_as(C.POINTER(C.c_int32)),
                                    len(out)), "pam_plan_get_bins")
    return out


def pam_workspace_size(plan: Plan, n_frames: int, n_t: Optional[int] = None) -> int:
    n = C.c_size_t()
    n_t = plan.info.n_samples if n_t is None else n_t
    _check(_lib().pam_workspace_size(C.c_void_p(plan.handle), n_frames, n_t, C.byref(n)), "pam_workspace_size")
    return n.value


def pam_workspace_layout(plan: Plan, n_frames: int, n_t: Optional[int] = None) -> LayoutC:
    lay = LayoutC()
    n_t = plan.info.n_samples if n_t is None else n_t
    _check(_lib().pam_workspace_layout(C.c_void_p(plan.handle), n_frames, n_t, C.byref(lay)),
           "pam_workspace_layout")
    return lay


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def check_buffers(info, rf, image, nncc=None, rho_pairs=None, workspace=None, n_t=None) -> None:
    """Reject buffers the C-ABI cannot check itself (it sees raw pointers): every tensor must
    be a contiguous tensor on the plan's GPU, rf float32 [F][L][n_t], image and nncc float32
    [F][n_z][N_x], rho_pairs float32 [F][n_pairs][n_z][N_x].  Raises PamError before any launch."""
    import torch

    def bad(msg):
        raise PamError(PAM_ERR_INVALID_ARG, f"pam_as_tax: {msg}")

    if rf is None or image is None:
        bad("rf and image are required")
    if rf.dim() != 3:
        bad(f"rf must be [F][L][n_t], got shape {tuple(rf.shape)}")
    F = int(rf.shape[0])
    n_t = int(rf.shape[-1]) if n_t is None else int(n_t)
    want = {"rf": (rf, (F, info.n_elements, n_t)), "image": (image, (F, info.n_z, info.n_x))}
    if nncc is not None:
        want["nncc"] = (nncc, (F, info.n_z, info.n_x))
    if rho_pairs is not None:
        want["rho_pairs"] = (rho_pairs, (F, info.n_pairs, info.n_z, info.n_x))
    for name, (t, shape) in want.items():
        if t.dtype != torch.float32:
            bad(f"{name} must be float32, got {t.dtype}")
        if tuple(t.shape) != shape:
            bad(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    tensors = [t for t, _ in want.values()] + ([workspace] if workspace is not None else [])
    for t in tensors:
        if not t.is_contiguous():
            bad("every buffer must be contiguous")
        if t.device.type != "cuda" or t.device.index != info.device:
            bad(f"every buffer must live on cuda:{info.device}, got {t.device}")


def pam_as_tax(plan: Plan, rf, image, nncc=None, rho_pairs=None, workspace=None, stream=None,
               n_t: Optional[int] = None) -> None:
    """Enqueue one reconstruction of rf [F][L][n_t] (device float32) on `stream`."""
    import torch
    F = int(rf.shape[0])
    n_t = int(rf.shape[-1]) if n_t is None else n_t
    check_buffers(plan.info, rf, image, nncc, rho_pairs, workspace, n_t)
    if stream is None:
        stream = torch.cuda.current_stream(rf.device)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    st = _lib().pam_as_tax(C.c_void_p(plan.handle), _ptr(rf), F, n_t, _ptr(image), _ptr(nncc),
                           _ptr(rho_pairs), _ptr(workspace), ws_bytes, C.c_void_p(stream.cuda_stream))
    _check(st, "pam_as_tax")


def pam_fd_tea_tax(plan: Plan, rf, image, nncc=None, rho_pairs=None, workspace=None, stream=None,
                   n_t: Optional[int] = None) -> None:
    """Frequency-domain delay-and-sum with the same weighting (FD-TEA-TAX) on the same plan."""
    import torch
    F = int(rf.shape[0])
    n_t = int(rf.shape[-1]) if n_t is None else n_t
    check_buffers(plan.info, rf, image, nncc, rho_pairs, workspace, n_t)
    if stream is None:
        stream = torch.cuda.current_stream(rf.device)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    st = _lib().pam_fd_tea_tax(C.c_void_p(plan.handle), _ptr(rf), F, n_t, _ptr(image), _ptr(nncc),
                               _ptr(rho_pairs), _ptr(workspace), ws_bytes, C.c_void_p(stream.cuda_stream))
    _check(st, "pam_fd_tea_tax")


NOALLOC_SCRATCH_BYTES = 128 << 20


def pam_as_tax_noalloc(plan: Plan, rf, image, nncc=None, rho_pairs=None, stream=None,
                       n_t: Optional[int] = None) -> None:
    """pam_as_tax on the library's built-in device scratch (no workspace, no allocation)."""
    import torch
    F = int(rf.shape[0])
    n_t = int(rf.shape[-1]) if n_t is None else n_t
    check_buffers(plan.info, rf, image, nncc, rho_pairs, None, n_t)
    if stream is None:
        stream = torch.cuda.current_stream(rf.device)
    st = _lib().pam_as_tax_noalloc(C.c_void_p(plan.handle), _ptr(rf), F, n_t, _ptr(image), _ptr(nncc),
                                   _ptr(rho_pairs), C.c_void_p(stream.cuda_stream))
    _check(st, "pam_as_tax_noalloc")


N_STAGE_EVENTS = 5
STAGES = ("time_fft", "lateral", "fields", "finalize")


def pam_as_tax_events(plan: Plan, rf, image, events, nncc=None, rho_pairs=None, workspace=None,
                      stream=None, n_t: Optional[int] = None) -> None:
    """pam_as_tax recording N_STAGE_EVENTS raw hipEvent_t handles at the stage boundaries."""
    import torch
    F = int(rf.shape[0])
    n_t = int(rf.shape[-1]) if n_t is None else n_t
    check_buffers(plan.info, rf, image, nncc, rho_pairs, workspace, n_t)
    if stream is None:
        stream = torch.cuda.current_stream(rf.device)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    arr = (C.c_void_p * N_STAGE_EVENTS)(*events)
    st = _lib().pam_as_tax_events(C.c_void_p(plan.handle), _ptr(rf), F, n_t, _ptr(image), _ptr(nncc),
                                  _ptr(rho_pairs), _ptr(workspace), ws_bytes,
                                  C.c_void_p(stream.cuda_stream), arr)
    _check(st, "pam_as_tax_events")


class HipEvents:
    """Raw HIP timing events from the process's HIP runtime (plumbing for timing only)."""

    def __init__(self):
        _lib()
        self.rt = C.CDLL("libamdhip64.so.7")
        self.rt.hipEventCreateWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_uint]
        self.rt.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.rt.hipEventDestroy.argtypes = [C.c_void_p]
        self.rt.hipEventSynchronize.argtypes = [C.c_void_p]
        self.live = []

    def create(self, n: int):
        out = []
        for _ in range(n):
            e = C.c_void_p()
            if self.rt.hipEventCreateWithFlags(C.byref(e), 0) != 0:
                raise RuntimeError("hipEventCreateWithFlags failed")
            out.append(e.value)
        self.live += out
        return out

    def elapsed_ms(self, a, b) -> float:
        ms = C.c_float()
        if self.rt.hipEventElapsedTime(C.byref(ms), C.c_void_p(a), C.c_void_p(b)) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def close(self):
        for e in self.live:
            self.rt.hipEventDestroy(C.c_void_p(e))
        self.live = []


def alloc_workspace(plan: Plan, n_frames: int, n_t: Optional[int] = None, device="cuda"):
    import torch
    n = pam_workspace_size(plan, n_frames, n_t)
    return torch.empty(n, dtype=torch.uint8, device=device)


def reconstruct(plan: Plan, rf, want_nncc=True, want_pairs=False, workspace=None, stream=None):
    """Allocate outputs (and a workspace if none is given), run pam_as_tax, return a dict."""
    import torch
    F, n_t = int(rf.shape[0]), int(rf.shape[-1])
    dev = rf.device
    out = {"image": torch.empty((F, plan.n_z, plan.n_x), dtype=torch.float32, device=dev)}
    out["nncc"] = torch.empty_like(out["image"]) if want_nncc else None
    out["rho_pairs"] = (torch.empty((F, plan.n_pairs, plan.n_z, plan.n_x), dtype=torch.float32, device=dev)
                        if want_pairs and plan.n_pairs else None)
    ws = alloc_workspace(plan, F, n_t, dev) if workspace is None else workspace
    pam_as_tax(plan, rf, out["image"], out["nncc"], out["rho_pairs"], ws, stream, n_t)
    out["workspace"] = ws
    return out
