"""Python binding of libcfog (ctypes).  Argument marshalling only: every step
of extraction and matching runs in the library's HIP kernels.  PyTorch is used
for device memory and streams.

    import torch
    from paper_1808_06194_amd import cfog
    vol, sat = cfog.cfog_extract(img)                      # img: cuda fp32 (H, W)
    res = cfog.match_batch([cfog.Job(volA, satA, volB, satB, cps, N=48, r=10)])
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcfog.so")

CFOG_OK = 0
CFOG_EINVAL = -1
CFOG_EUNSUPPORTED = -2
CFOG_ENOMEM = -3
CFOG_EHIP = -4

CP_OK, CP_OUT_OF_BOUNDS, CP_NONFINITE = 0, 1, 2

PATH_PLAIN_FFT = 0x1
PATH_BATCHED_FFT = 0x2
PATH_MFMA_BF16 = 0x4
AUTOTUNE = 0x100
USE_GRAPH = 0x200
OBJ_CORR = 0x400
NO_SPLIT = 0x800

# Exported symbols, as declared in include/cfog.h.
EXPORTS = (
    "cfog_ctx_create", "cfog_ctx_destroy", "cfog_ctx_last_error", "cfog_status_str",
    "cfog_extract", "cfog_extract_scheme", "cfog_extract_fhog", "cfog_extract_workspace_size",
    "cfog_extract_batch_workspace_size", "cfog_extract_batch", "match_batch_workspace_size", "match_batch",
    "cfog_max_window", "cfog_fft_size", "cfog_set_plan", "cfog_plan_for", "cfog_harris_grid",
    "cfog_reject_outliers",
    "cfog_server_create", "cfog_server_destroy", "cfog_server_add_pair", "cfog_server_submit",
    "cfog_server_poll", "cfog_server_get_stats", "match_batch_noalloc", "cfog_noalloc_scratch_bytes",
)


class CfogError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_str(code)} ({code})")
        self.code = code


class cfog_job(ctypes.Structure):
    _fields_ = [
        ("volA", ctypes.c_void_p), ("satA", ctypes.c_void_p), ("hA", ctypes.c_int32), ("wA", ctypes.c_int32),
        ("volB", ctypes.c_void_p), ("satB", ctypes.c_void_p), ("hB", ctypes.c_int32), ("wB", ctypes.c_int32),
        ("cps", ctypes.c_void_p), ("n_cps", ctypes.c_int32), ("N", ctypes.c_int32), ("r", ctypes.c_int32),
        ("pad_", ctypes.c_int32), ("out", ctypes.c_void_p), ("surfaces", ctypes.c_void_p),
        ("subpix", ctypes.c_void_p),
    ]


class cfog_image(ctypes.Structure):
    _fields_ = [
        ("d_img", ctypes.c_void_p), ("row_stride", ctypes.c_int64), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
        ("d_vol", ctypes.c_void_p), ("d_sat", ctypes.c_void_p),
    ]


class cfog_reject_result(ctypes.Structure):
    _fields_ = [
        ("coef", (ctypes.c_double * 2) * 10), ("centre", ctypes.c_double * 2), ("half_extent", ctypes.c_double * 2),
        ("rmse", ctypes.c_double), ("removed", ctypes.c_int32), ("n_kept", ctypes.c_int32),
        ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
    ]


class cfog_server_config(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t), ("n_slots", ctypes.c_int32), ("max_batch_cps", ctypes.c_int32),
        ("max_batch_reqs", ctypes.c_int32), ("m", ctypes.c_int32), ("sigma", ctypes.c_float),
        ("flags", ctypes.c_int32), ("max_batch_surf", ctypes.c_size_t),
    ]


class cfog_request_info(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64), ("status", ctypes.c_int32), ("n_cps", ctypes.c_int32),
        ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64), ("t_launch_ns", ctypes.c_int64),
        ("t_done_ns", ctypes.c_int64), ("batch_reqs", ctypes.c_int32), ("pad", ctypes.c_int32),
    ]


class cfog_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
        ("evictions", ctypes.c_int64), ("extractions", ctypes.c_int64), ("blocked", ctypes.c_int64),
        ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t),
        ("max_in_flight", ctypes.c_int32), ("pad", ctypes.c_int32),
    ]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libcfog.so (built in-tree by paper_1808_06194_amd.build).  Raises
    if it is missing: there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing; build it with `python -m paper_1808_06194_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.cfog_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.cfog_ctx_destroy.argtypes = [vp]
    lib.cfog_ctx_last_error.argtypes = [vp]
    lib.cfog_status_str.argtypes = [ctypes.c_int]
    lib.cfog_status_str.restype = ctypes.c_char_p
    lib.cfog_extract.argtypes = [vp, vp, i32, i32, i64, i32, ctypes.c_float, i32, vp, vp, vp, sz, vp]
    lib.cfog_extract_scheme.argtypes = [vp, vp, i32, i32, i64, i32, ctypes.c_float, i32, i32, vp, vp, vp, sz, vp]
    lib.cfog_extract_fhog.argtypes = [vp, vp, i32, i32, i64, i32, vp, vp, vp, sz, vp]
    lib.cfog_extract_workspace_size.argtypes = [i32, i32]
    lib.cfog_extract_workspace_size.restype = sz
    lib.cfog_extract_batch_workspace_size.argtypes = [ctypes.POINTER(cfog_image), i32]
    lib.cfog_extract_batch_workspace_size.restype = sz
    lib.cfog_extract_batch.argtypes = [vp, ctypes.POINTER(cfog_image), i32, i32, ctypes.c_float, i32, i32, vp, sz, vp]
    lib.match_batch_workspace_size.argtypes = [vp, ctypes.POINTER(cfog_job), i32, i32, i32]
    lib.match_batch_workspace_size.restype = sz
    lib.match_batch.argtypes = [vp, ctypes.POINTER(cfog_job), i32, i32, i32, vp, sz, vp]
    lib.match_batch_noalloc.argtypes = [vp, ctypes.POINTER(cfog_job), i32, i32, i32, vp]
    lib.cfog_noalloc_scratch_bytes.restype = sz
    lib.cfog_max_window.restype = i32
    lib.cfog_fft_size.argtypes = [i32, i32]
    lib.cfog_fft_size.restype = i32
    lib.cfog_set_plan.argtypes = [vp, i32, i32, i32]
    lib.cfog_plan_for.argtypes = [vp, i32, i32, i32]
    lib.cfog_plan_for.restype = i32
    lib.cfog_harris_grid.argtypes = [vp, vp, i32, i32, i64, i32, i32, i32, ctypes.c_float, ctypes.c_float, vp, vp, vp]
    lib.cfog_reject_outliers.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp, vp]
    lib.cfog_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(cfog_server_config), ctypes.POINTER(vp)]
    lib.cfog_server_destroy.argtypes = [vp]
    lib.cfog_server_add_pair.argtypes = [vp, vp, i32, i32, i64, vp, i32, i32, i64, ctypes.POINTER(i32)]
    lib.cfog_server_submit.argtypes = [vp, i32, vp, i32, i32, i32, vp, vp, ctypes.POINTER(i64)]
    lib.cfog_server_poll.argtypes = [vp, ctypes.POINTER(cfog_request_info), i32, i64, ctypes.POINTER(i32)]
    lib.cfog_server_get_stats.argtypes = [vp, ctypes.POINTER(cfog_server_stats)]
    _lib = lib
    return lib


def status_str(code: int) -> str:
    return load().cfog_status_str(int(code)).decode()


def _check(code: int, what: str):
    if code != CFOG_OK:
        raise CfogError(code, what)


class Context:
    """A libcfog context bound to one HIP device."""

    def __init__(self, device: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.cfog_ctx_create(int(device), ctypes.byref(h)), "cfog_ctx_create")
        self.handle = h
        self.device = device
        self._ws = None

    def close(self):
        if self.handle:
            load().cfog_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> int:
        return load().cfog_ctx_last_error(self.handle)

    def workspace(self, nbytes: int) -> torch.Tensor:
        """Context-cached device workspace of at least nbytes."""
        if nbytes <= 0:
            return None
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws


_ctx: dict = {}


def context(device: Optional[int] = None) -> Context:
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _ctx:
        _ctx[dev] = Context(dev)
    return _ctx[dev]


def _stream_ptr(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_out(t: Optional[torch.Tensor], shape, dtype, like: torch.Tensor, what: str):
    """A caller-supplied output must have exactly the layout the library
    writes: shape, dtype, contiguous, on the image's device."""
    if t is None:
        return
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_contiguous() or t.device != like.device:
        raise ValueError(f"{what} must be a contiguous {dtype} tensor of shape {tuple(shape)} on {like.device}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device} (contiguous={t.is_contiguous()})")


def _check_workspace(ws: Optional[torch.Tensor], need: int, what: str):
    if ws is None:
        return
    if ws.dtype != torch.uint8 or not ws.is_cuda or not ws.is_contiguous() or ws.numel() < need:
        raise ValueError(f"{what}: workspace must be a contiguous cuda uint8 tensor of >= {need} bytes")


def extract_workspace_size(H: int, W: int) -> int:
    return int(load().cfog_extract_workspace_size(int(H), int(W)))


def cfog_extract(img: torch.Tensor, m: int = 9, sigma: float = 0.8, radius: int = -1, with_sat: bool = True,
                 vol: Optional[torch.Tensor] = None, sat: Optional[torch.Tensor] = None, stream=None,
                 workspace: Optional[torch.Tensor] = None, scheme: int = 2):
    """CFOG volume (m, H, W) fp32 and FP64 SAT (H+1, W+1) of a 2-D cuda fp32 image.
    `workspace` (uint8 cuda tensor of >= extract_workspace_size(H, W) bytes) is
    needed only when extractions on several streams overlap.  scheme 2: the
    oriented channels of Eq. 2; scheme 1: binned orientation."""
    if img.dim() != 2 or img.dtype != torch.float32 or not img.is_cuda or img.stride(1) != 1:
        raise ValueError("img must be a 2-D row-contiguous cuda float32 tensor")
    H, W = img.shape
    _check_out(vol, (m, H, W), torch.float32, img, "vol")
    _check_out(sat if with_sat else None, (H + 1, W + 1), torch.float64, img, "sat")
    if vol is None:
        vol = torch.empty((m, H, W), dtype=torch.float32, device=img.device)
    if with_sat and sat is None:
        sat = torch.empty((H + 1, W + 1), dtype=torch.float64, device=img.device)
    if with_sat:
        _check_workspace(workspace, extract_workspace_size(H, W), "cfog_extract")
    ctx = context(img.device.index)
    rc = load().cfog_extract_scheme(ctx.handle, img.data_ptr(), H, W, img.stride(0), m, float(sigma), int(radius),
                                    int(scheme), vol.data_ptr(), _ptr(sat) if with_sat else None, _ptr(workspace),
                                    workspace.numel() if workspace is not None else 0, _stream_ptr(stream))
    _check(rc, "cfog_extract")
    return vol, (sat if with_sat else None)


def _image_array(imgs, vols, sats):
    arr = (cfog_image * max(1, len(imgs)))()
    for i, (img, vol, sat) in enumerate(zip(imgs, vols, sats)):
        arr[i] = cfog_image(img.data_ptr(), img.stride(0), img.shape[0], img.shape[1], vol.data_ptr(), _ptr(sat))
    return arr


def extract_batch_workspace_size(shapes, with_sat: bool = True) -> int:
    """Workspace bytes of cfog_extract_batch for images of the given (H, W)."""
    arr = (cfog_image * max(1, len(shapes)))()
    for i, (H, W) in enumerate(shapes):
        arr[i] = cfog_image(None, W, H, W, None, 8 if with_sat else None)  # only the sizes and SAT presence count
    return int(load().cfog_extract_batch_workspace_size(arr, len(shapes)))


def cfog_extract_batch(imgs, m: int = 9, sigma: float = 0.8, radius: int = -1, with_sat: bool = True,
                       vols=None, sats=None, stream=None, workspace: Optional[torch.Tensor] = None, scheme: int = 2):
    """cfog_extract of several 2-D cuda fp32 images (same parameters) in one
    call: lists of volumes (m, H, W) and SATs (H+1, W+1) (None without SATs)."""
    for img in imgs:
        if img.dim() != 2 or img.dtype != torch.float32 or not img.is_cuda or img.stride(1) != 1:
            raise ValueError("every image must be a 2-D row-contiguous cuda float32 tensor")
    if vols is None:
        vols = [torch.empty((m, *img.shape), dtype=torch.float32, device=img.device) for img in imgs]
    if not with_sat:
        sats = [None] * len(imgs)
    elif sats is None:
        sats = [torch.empty((img.shape[0] + 1, img.shape[1] + 1), dtype=torch.float64, device=img.device)
                for img in imgs]
    if len(vols) != len(imgs) or len(sats) != len(imgs):
        raise ValueError("cfog_extract_batch: one volume (and SAT) per image")
    for i, (img, vol, sat) in enumerate(zip(imgs, vols, sats)):  # a None SAT: that image gets none
        H, W = img.shape
        _check_out(vol, (m, H, W), torch.float32, img, f"vols[{i}]")
        _check_out(sat, (H + 1, W + 1), torch.float64, img, f"sats[{i}]")
    arr = _image_array(imgs, vols, sats)
    _check_workspace(workspace, int(load().cfog_extract_batch_workspace_size(arr, len(imgs))), "cfog_extract_batch")
    ctx = context(imgs[0].device.index if len(imgs) else None)
    rc = load().cfog_extract_batch(ctx.handle, arr, len(imgs), m, float(sigma), int(radius), int(scheme),
                                   _ptr(workspace), workspace.numel() if workspace is not None else 0,
                                   _stream_ptr(stream))
    _check(rc, "cfog_extract_batch")
    return vols, (sats if with_sat else None)


FHOG_CHANNELS = 36


def fhog_extract(img: torch.Tensor, cell: int = 4, with_sat: bool = True, vol: Optional[torch.Tensor] = None,
                 sat: Optional[torch.Tensor] = None, stream=None, workspace: Optional[torch.Tensor] = None):
    """Pixel-wise HOG volume (36, H, W) fp32 (2 x 2 cells of `cell` pixels,
    9 unsigned bins) and its FP64 SAT; match it with match_batch(m=36)."""
    if img.dim() != 2 or img.dtype != torch.float32 or not img.is_cuda or img.stride(1) != 1:
        raise ValueError("img must be a 2-D row-contiguous cuda float32 tensor")
    H, W = img.shape
    _check_out(vol, (FHOG_CHANNELS, H, W), torch.float32, img, "vol")
    _check_out(sat if with_sat else None, (H + 1, W + 1), torch.float64, img, "sat")
    if with_sat:
        _check_workspace(workspace, extract_workspace_size(H, W), "fhog_extract")
    if vol is None:
        vol = torch.empty((FHOG_CHANNELS, H, W), dtype=torch.float32, device=img.device)
    if with_sat and sat is None:
        sat = torch.empty((H + 1, W + 1), dtype=torch.float64, device=img.device)
    ctx = context(img.device.index)
    rc = load().cfog_extract_fhog(ctx.handle, img.data_ptr(), H, W, img.stride(0), int(cell), vol.data_ptr(),
                                  _ptr(sat) if with_sat else None, _ptr(workspace),
                                  workspace.numel() if workspace is not None else 0, _stream_ptr(stream))
    _check(rc, "cfog_extract_fhog")
    return vol, (sat if with_sat else None)


@dataclasses.dataclass
class Job:
    """One matching job: volumes + SATs of A and B, control points (n, 4) int32
    cuda tensor of (x, y, bx, by), template side N, search radius r."""
    volA: torch.Tensor
    satA: torch.Tensor
    volB: torch.Tensor
    satB: torch.Tensor
    cps: torch.Tensor
    N: int
    r: int
    out: Optional[torch.Tensor] = None        # (n, 6) int32 view of cfog_result
    surfaces: Optional[torch.Tensor] = None   # (n, 2r+1, 2r+1) fp32
    subpix: Optional[torch.Tensor] = None     # (n, 2) fp32 refined offsets (fdx, fdy)

    def to_c(self) -> cfog_job:
        n = int(self.cps.shape[0])
        if self.out is None:
            self.out = torch.empty((n, 6), dtype=torch.int32, device=self.cps.device)
        return cfog_job(
            self.volA.data_ptr(), self.satA.data_ptr(), self.volA.shape[1], self.volA.shape[2],
            self.volB.data_ptr(), self.satB.data_ptr(), self.volB.shape[1], self.volB.shape[2],
            self.cps.data_ptr() if n else None, n, int(self.N), int(self.r), 0,
            self.out.data_ptr(), _ptr(self.surfaces), _ptr(self.subpix))


def results(out: torch.Tensor) -> dict:
    """Split an (n, 6) int32 result tensor into named fields (on its device)."""
    return dict(dx=out[:, 0], dy=out[:, 1], best=out[:, 2].view(torch.float32),
                second=out[:, 3].view(torch.float32), status=out[:, 4])


def make_jobs_array(jobs: List[Job]):
    arr = (cfog_job * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        arr[i] = j.to_c()
    return arr


def match_batch(jobs: List[Job], m: int = 9, flags: int = PATH_PLAIN_FFT, stream=None,
                workspace: Optional[torch.Tensor] = None, ctx: Optional["Context"] = None) -> List[torch.Tensor]:
    """Match every control point of every job; returns the (n, 6) int32 result
    tensors (see `results`).  Asynchronous on `stream`.  Without an explicit
    `workspace` the context's cached one is used (grown on demand).  `ctx`:
    the context whose FFT-size choices (pins, autotuned picks) apply; by
    default the device's shared one."""
    if not jobs:
        return []
    dev = jobs[0].cps.device.index
    ctx = context(dev) if ctx is None else ctx
    arr = make_jobs_array(jobs)
    lib = load()
    for attempt in range(2):
        need = lib.match_batch_workspace_size(ctx.handle, arr, len(jobs), m, flags)
        if need == ctypes.c_size_t(-1).value:
            raise CfogError(CFOG_EINVAL, "match_batch_workspace_size")
        ws = workspace if workspace is not None else ctx.workspace(need)
        rc = lib.match_batch(ctx.handle, arr, len(jobs), m, flags, _ptr(ws) if need else None,
                             ws.numel() if (need and ws is not None) else 0, _stream_ptr(stream))
        # an autotuning call may have picked a larger FFT size: query again
        if rc == CFOG_ENOMEM and workspace is None and attempt == 0:
            continue
        break
    _check(rc, "match_batch")
    return [j.out for j in jobs]


def match_batch_noalloc(jobs: List[Job], m: int = 9, flags: int = PATH_PLAIN_FFT, stream=None) -> List[torch.Tensor]:
    """match_batch through the entry point that allocates nothing (its
    workspace is the library's static device array; see match_batch_noalloc
    in include/cfog.h).  The jobs' result tensors must already exist: this
    wrapper allocates nothing either."""
    if not jobs:
        return []
    for j in jobs:
        if j.out is None or tuple(j.out.shape) != (int(j.cps.shape[0]), 6) or j.out.dtype != torch.int32:
            raise ValueError("match_batch_noalloc: every job needs its (n, 6) int32 `out` tensor")
    ctx = context(jobs[0].cps.device.index)
    arr = make_jobs_array(jobs)
    _check(load().match_batch_noalloc(ctx.handle, arr, len(jobs), m, flags, _stream_ptr(stream)),
           "match_batch_noalloc")
    return [j.out for j in jobs]


def harris_grid(img: torch.Tensor, n: int, k: int, chip: int = 60, sigma: float = 1.0, kappa: float = 0.04,
                stream=None):
    """Block-based Harris feature points of a 2-D cuda fp32 image (see
    cfog_harris_grid in include/cfog.h).  Returns (cps (n*n*k, 4) int32 cuda
    tensor of (x, y, x, y), responses (n*n*k,) fp32), asynchronously."""
    if img.dim() != 2 or img.dtype != torch.float32 or not img.is_cuda or img.stride(1) != 1:
        raise ValueError("img must be a 2-D row-contiguous cuda float32 tensor")
    H, W = img.shape
    cps = torch.empty((n * n * k, 4), dtype=torch.int32, device=img.device)
    resp = torch.empty((n * n * k,), dtype=torch.float32, device=img.device)
    rc = load().cfog_harris_grid(context(img.device.index).handle, img.data_ptr(), H, W, img.stride(0), int(n),
                                 int(k), int(chip), float(sigma), float(kappa), cps.data_ptr(), resp.data_ptr(),
                                 _stream_ptr(stream))
    _check(rc, "cfog_harris_grid")
    return cps, resp


def reject_outliers(src: torch.Tensor, dst: torch.Tensor, threshold: float = 3.5, stream=None,
                    keep: Optional[torch.Tensor] = None, result: Optional[torch.Tensor] = None, sync: bool = True):
    """Iterative cubic-polynomial outlier rejection (see cfog_reject_outliers
    in include/cfog.h).  src, dst: (n, 2) cuda fp32 point coordinates.
    keep / result: optional preallocated outputs ((n,) uint8; a cuda tensor of
    at least 216 bytes, 8-byte aligned).  Returns (keep, result dict with coef
    (10, 2), centre, half_extent, rmse, removed, n_kept, status) after
    synchronising, or (keep, result tensor) with sync=False."""
    if src.shape != dst.shape or src.dim() != 2 or src.shape[1] != 2:
        raise ValueError("src and dst must be (n, 2)")
    src = src.to(torch.float32).contiguous()
    dst = dst.to(torch.float32).contiguous()
    n = src.shape[0]
    if keep is None:
        keep = torch.empty((n,), dtype=torch.uint8, device=src.device)
    if result is None:
        result = torch.empty((ctypes.sizeof(cfog_reject_result),), dtype=torch.uint8, device=src.device)
    if keep.numel() < n or result.numel() * result.element_size() < ctypes.sizeof(cfog_reject_result):
        raise ValueError("keep or result too small")
    rc = load().cfog_reject_outliers(context(src.device.index).handle, src.data_ptr(), dst.data_ptr(), n,
                                     float(threshold), keep.data_ptr(), result.data_ptr(), _stream_ptr(stream))
    _check(rc, "cfog_reject_outliers")
    if not sync:
        return keep, result
    torch.cuda.synchronize(src.device)
    return keep, reject_result_dict(result)


def reject_result_dict(result: torch.Tensor) -> dict:
    """The fields of a cfog_reject_result held in a device or host tensor."""
    raw = result.contiguous().view(torch.uint8).cpu().numpy().tobytes()[:ctypes.sizeof(cfog_reject_result)]
    r = cfog_reject_result.from_buffer_copy(raw)
    import numpy as np
    return dict(coef=np.array([[r.coef[a][c] for c in range(2)] for a in range(10)]),
                centre=np.array(list(r.centre)), half_extent=np.array(list(r.half_extent)), rmse=r.rmse,
                removed=r.removed, n_kept=r.n_kept, status=r.status)


def set_plan(N: int, r: int, P: int, device: Optional[int] = None):
    """Pin the FFT side used for (N, r) on the device's context (0 unpins)."""
    _check(load().cfog_set_plan(context(device).handle, int(N), int(r), int(P)), "cfog_set_plan")


def plan_for(N: int, r: int, m: int = 9, device: Optional[int] = None) -> int:
    return int(load().cfog_plan_for(context(device).handle, int(N), int(r), int(m)))


def max_window() -> int:
    return int(load().cfog_max_window())


def fft_size(N: int, r: int) -> int:
    """FFT side P used for template side N and radius r (0 if unsupported)."""
    return int(load().cfog_fft_size(int(N), int(r)))


# ------------------------------------------------------------------ serving

@dataclasses.dataclass
class Completed:
    """A finished server request: results (n, 6) int32 host array (see
    `results_np`), optional surfaces (n, 2r+1, 2r+1) fp32, status and
    CLOCK_MONOTONIC timestamps in ns (same clock as time.monotonic_ns)."""
    id: int
    status: int
    out: "np.ndarray"
    surfaces: Optional["np.ndarray"]
    t_submit: int
    t_admit: int
    t_launch: int
    t_done: int
    batch_reqs: int


def results_np(out) -> dict:
    """Split an (n, 6) int32 host result array into named fields."""
    return dict(dx=out[:, 0], dy=out[:, 1], best=out[:, 2].view("float32"),
                second=out[:, 3].view("float32"), status=out[:, 4])


class Server:
    """Matching server: resident CFOG volumes of registered pairs, admission by
    device memory, continuous batching over `n_slots` streams (see the serving
    section of include/cfog.h).  Images passed to add_pair stay referenced here
    for the server's lifetime."""

    def __init__(self, hbm_budget: int, n_slots: int = 4, max_batch_cps: int = 8192, max_batch_reqs: int = 256,
                 m: int = 9, sigma: float = 0.8, flags: int = PATH_BATCHED_FFT, max_batch_surf: int = 1 << 22,
                 device: int = 0):
        lib = load()
        cfg = cfog_server_config(int(hbm_budget), int(n_slots), int(max_batch_cps), int(max_batch_reqs), int(m),
                                 float(sigma), int(flags), int(max_batch_surf))
        h = ctypes.c_void_p()
        _check(lib.cfog_server_create(int(device), ctypes.byref(cfg), ctypes.byref(h)), "cfog_server_create")
        self.handle = h
        self._images = []
        self._live = {}   # id -> (out, surfaces, cps) host arrays kept alive until reported

    def close(self):
        if self.handle:
            load().cfog_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def add_pair(self, imgA: torch.Tensor, imgB: torch.Tensor) -> int:
        for t in (imgA, imgB):
            if t.dim() != 2 or t.dtype != torch.float32 or not t.is_cuda or t.stride(1) != 1:
                raise ValueError("images must be 2-D row-contiguous cuda float32 tensors")
        pid = ctypes.c_int32()
        _check(load().cfog_server_add_pair(self.handle, imgA.data_ptr(), imgA.shape[0], imgA.shape[1],
                                           imgA.stride(0), imgB.data_ptr(), imgB.shape[0], imgB.shape[1],
                                           imgB.stride(0), ctypes.byref(pid)), "cfog_server_add_pair")
        self._images.append((imgA, imgB))
        return pid.value

    def submit(self, pair: int, cps, N: int, r: int, surfaces: bool = False) -> int:
        """Submit control points `cps` ((n, 4) int32 array-like of x, y, bx, by)."""
        import numpy as np
        c = np.ascontiguousarray(np.asarray(cps, dtype=np.int32).reshape(-1, 4))
        n = c.shape[0]
        out = np.zeros((n, 6), np.int32)
        K = 2 * int(r) + 1
        surf = np.zeros((n, K, K), np.float32) if surfaces else None
        rid = ctypes.c_int64()
        _check(load().cfog_server_submit(self.handle, int(pair), c.ctypes.data, n, int(N), int(r),
                                         out.ctypes.data, surf.ctypes.data if surf is not None else None,
                                         ctypes.byref(rid)), "cfog_server_submit")
        self._live[rid.value] = (out, surf)
        return rid.value

    def poll(self, max_n: int = 1024, timeout_us: int = 0) -> List[Completed]:
        infos = (cfog_request_info * max(1, max_n))()
        n = ctypes.c_int32()
        _check(load().cfog_server_poll(self.handle, infos, int(max_n), int(timeout_us), ctypes.byref(n)),
               "cfog_server_poll")
        done = []
        for i in range(n.value):
            f = infos[i]
            out, surf = self._live.pop(f.id)
            done.append(Completed(f.id, f.status, out, surf, f.t_submit_ns, f.t_admit_ns, f.t_launch_ns,
                                  f.t_done_ns, f.batch_reqs))
        return done

    def wait(self, ids, timeout_s: float = 60.0) -> dict:
        """Poll until every id in `ids` is reported; returns {id: Completed}."""
        import time
        want, got = set(ids), {}
        t_end = time.monotonic() + timeout_s
        while want - got.keys():
            if time.monotonic() > t_end:
                raise TimeoutError(f"{len(want - got.keys())} requests still pending")
            for c in self.poll(timeout_us=10000):
                got[c.id] = c
        return got

    def stats(self) -> dict:
        st = cfog_server_stats()
        _check(load().cfog_server_get_stats(self.handle, ctypes.byref(st)), "cfog_server_get_stats")
        return {k: getattr(st, k) for k, _ in cfog_server_stats._fields_ if k != "pad"}
