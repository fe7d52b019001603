"""Python front end of libdwt2: tensors in, tensors out.

Every call marshals device pointers, strides and the current HIP stream into
the C ABI; all arithmetic runs in the library's HIP kernels.  Tensors must
live on a ROCm device, be float32 (DWT2_F32) or int32 (DWT2_I32_REV), and have
unit stride along the last (width) axis.
"""
from __future__ import annotations

import ctypes
from collections import OrderedDict
from typing import List, Sequence

import torch

from . import _lib
from ._lib import DWT2_EXT_SYMMETRIC, DWT2_F32, DWT2_I32_REV

__all__ = ["fwd", "inv", "bwd", "fwd_batched", "inv_batched", "bwd_batched", "DWT2Function", "workspace_size",
           "batched_workspace_size", "level_sizes", "set_tiling", "set_path", "set_probe", "fwd_separable",
           "separable_workspace_size", "fwd_lds", "fwd_cdf97", "inv_cdf97", "fwd_cdf97_separable",
           "synchronize", "set_job_wait", "plan_cache_size", "launch_levels", "clear_plan_cache", "DWT2_F32", "DWT2_I32_REV"]


def level_sizes(w: int, h: int, levels: int):
    out = [(w, h)]
    for _ in range(levels):
        w, h = (w + 1) // 2, (h + 1) // 2
        out.append((w, h))
    return out


def _mode_of(t: torch.Tensor, mode) -> int:
    if mode is None:
        if t.dtype == torch.float32:
            return DWT2_F32
        if t.dtype == torch.int32:
            return DWT2_I32_REV
        raise TypeError(f"unsupported dtype {t.dtype}: float32 or int32 expected")
    want = torch.float32 if mode == DWT2_F32 else torch.int32
    if t.dtype != want:
        raise TypeError(f"mode {mode} needs {want}, got {t.dtype}")
    return mode


def _as_batch(t: torch.Tensor):
    """View (..., H, W) as (B, H, W) with uniform strides, copying if needed."""
    if not t.is_cuda:
        raise ValueError("the DWT runs on the GPU: move the tensor to a ROCm device first")
    if t.dim() < 2:
        raise ValueError("need at least (H, W)")
    h, w = t.shape[-2], t.shape[-1]
    b = t.reshape(-1, h, w) if t.dim() > 2 else t.unsqueeze(0)
    if b.stride(-1) != 1 or b.stride(-2) < w:
        b = b.contiguous()
    if b.shape[0] > 1 and b.stride(0) < b.stride(-2) * h:
        b = b.contiguous()
    return b


def set_tiling(seg: int = 0, chunk: int = 0) -> None:
    """Process-wide tiling override (0 = automatic); results do not change."""
    _lib.check(_lib.load().dwt2_set_tiling(seg, chunk))


PATHS = {"levels": 0, "persistent": 1, "levels-only": 2, "pairs": 3, "pairs-only": 4, "no-pairs": 5}


def set_path(path="levels") -> None:
    """How levels are chained (see dwt2_set_path): "levels" (default: pairs
    of levels in one launch for the inverse and adjoint, and for the forward
    where the pair's strips are at least 60 % filled or the level is small;
    the small coarsest levels fused into one launch where that saves a
    launch),
    "persistent" (one cooperative launch), "levels-only" (one launch per
    level throughout), "pairs" (pairs in every direction), "pairs-only"
    (pairs and single levels, no fused coarsest levels), "no-pairs" (single
    levels and the fused coarsest levels).  True / False select
    "persistent" / "levels".  Results are bit-identical."""
    if isinstance(path, bool):
        path = "persistent" if path else "levels"
    if path not in PATHS:
        raise ValueError(f"path must be one of {sorted(PATHS)}")
    _lib.check(_lib.load().dwt2_set_path(PATHS[path]))


_PROBE_DIRS = {"fwd": 0, "inv": 1, "bwd": 2}


def set_probe(direction: str | None, level: int = 1, begin: "torch.cuda.Event | None" = None,
              end: "torch.cuda.Event | None" = None) -> None:
    """Record `begin` / `end` (timing-enabled torch.cuda.Event) around the
    launch of `level` in every later `direction` call on the per-level path;
    `direction=None` clears the probe (see dwt2_set_probe)."""
    lib = _lib.load()
    if direction is None:
        _lib.check(lib.dwt2_set_probe(-1, 0, None, None))
        return
    if direction not in _PROBE_DIRS or begin is None or end is None:
        raise ValueError("direction must be 'fwd', 'inv' or 'bwd', with two events")
    for ev in (begin, end):
        if not ev.cuda_event:  # torch creates the HIP event on its first record
            ev.record()
    _lib.check(lib.dwt2_set_probe(_PROBE_DIRS[direction], level, begin.cuda_event, end.cuda_event))


def launch_levels(w: int, h: int, levels: int, direction: str = "fwd", batch: int = 1):
    """[(first, last), ...]: the launches of a plain call on the current path,
    in execution order, each with the levels it computes (dwt2_launch_levels)."""
    lib = _lib.load()
    first, last = (ctypes.c_int32 * 16)(), (ctypes.c_int32 * 16)()
    n = lib.dwt2_launch_levels(w, h, batch, levels, _PROBE_DIRS[direction], first, last, 16)
    _lib.check(min(n, 0))
    return [(first[i], last[i]) for i in range(n)]


def workspace_size(w: int, h: int, levels: int, batch: int = 1, mode: int = DWT2_F32) -> int:
    return int(_lib.load().dwt2_workspace_size(w, h, batch, levels, mode))


def _stream(device_index: int | None = None) -> int:
    """The raw handle of the current stream of `device_index` (default: the
    current device).  torch's raw-handle query takes about 0.3 us against
    3 us for building a Stream object, which matters for small calls."""
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return raw(torch.cuda.current_device() if device_index is None else device_index)
    if device_index is None:
        return torch.cuda.current_stream().cuda_stream
    return torch.cuda.current_stream(device_index).cuda_stream


def _geom(t: torch.Tensor):
    """(tensor, batch, h, w, row stride, batch stride) of (..., H, W) in
    elements, for the ABI.  A plain 2-D row-major view (the common small
    call) is taken as it is, without building a batched view; anything else
    goes through _as_batch."""
    if t.dim() == 2 and t.is_cuda and t.stride(1) == 1 and t.stride(0) >= t.shape[1]:
        return t, 1, t.shape[0], t.shape[1], t.stride(0), 0
    b = _as_batch(t)
    return b, b.shape[0], b.shape[1], b.shape[2], b.stride(1), b.stride(0) if b.shape[0] > 1 else 0


def fwd_separable(x: torch.Tensor, levels: int, mode=None, out=None, workspace=None) -> torch.Tensor:
    """The same forward transform by the separable lifting baseline (one
    kernel launch and one HBM pass per lifting step; see dwt2_fwd_separable).
    For comparisons, not for production use."""
    return _run("dwt2_fwd_separable", x, levels, mode, out, workspace)


def fwd_cdf97(x: torch.Tensor, levels: int, out=None, workspace=None) -> torch.Tensor:
    """Forward multi-level CDF 9/7 transform of float32 (..., H, W) by the
    non-separable scheme, one spatial predict and update per lifting pair
    (see dwt2_fwd_cdf97); Mallat-packed result of the same shape."""
    return _run("dwt2_fwd_cdf97", x, levels, None, out, workspace)


def fwd_cdf97_separable(x: torch.Tensor, levels: int, out=None, workspace=None) -> torch.Tensor:
    """The same CDF 9/7 forward by the separable comparison kernel (eight
    barrier-separated steps per level instead of four; see
    dwt2_fwd_cdf97_separable).  For comparisons, not for production use."""
    return _run("dwt2_fwd_cdf97_separable", x, levels, None, out, workspace)


def inv_cdf97(c: torch.Tensor, levels: int, out=None, workspace=None) -> torch.Tensor:
    """Inverse of fwd_cdf97."""
    return _run("dwt2_inv_cdf97", c, levels, None, out, workspace)


SCHEMES = {"separable": 0, "nonseparable": 1, "adapted": 2}


def fwd_lds(x: torch.Tensor, levels: int, scheme: str = "nonseparable", mode=None, out=None,
            workspace=None) -> torch.Tensor:
    """The same forward transform by the LDS-tiled comparison kernels
    (see dwt2_fwd_lds): scheme "separable" lifts each tile in four
    barrier-separated steps (eq. (3)), "nonseparable" in two (eq. (5)),
    "adapted" in two with the filters' constant terms applied separably
    (§3; float32 only).  For comparisons, not for production use."""
    if scheme not in SCHEMES:
        raise ValueError(f"scheme must be one of {sorted(SCHEMES)}")
    return _run("dwt2_fwd_lds", x, levels, mode, out, workspace, extra=(SCHEMES[scheme],))


def separable_workspace_size(w: int, h: int, levels: int, batch: int = 1, mode: int = DWT2_F32) -> int:
    return int(_lib.load().dwt2_separable_workspace_size(w, h, batch, levels, mode))


def _run(name: str, x: torch.Tensor, levels: int, mode, out: torch.Tensor | None,
         workspace: torch.Tensor | None = None, extra: tuple = (), lead: tuple = ()) -> torch.Tensor:
    lib = _lib.load()
    mode = _mode_of(x, mode)
    xb, batch, h, w, xs, xbs = _geom(x)
    if out is None:
        out = torch.empty(x.shape, dtype=x.dtype, device=x.device)
    ob, obatch, oh, ow, os_, obs = _geom(out)
    if (obatch, oh, ow) != (batch, h, w) or ob.dtype != xb.dtype:
        raise ValueError("out must match the input's shape and dtype")
    if ob.data_ptr() != out.data_ptr() or (out.dim() > 2 and not out.is_contiguous()):
        raise ValueError("out must be a contiguous tensor")
    size_fn = lib.dwt2_separable_workspace_size if name == "dwt2_fwd_separable" else lib.dwt2_workspace_size
    nbytes = int(size_fn(w, h, batch, levels, mode))
    ws = None
    if nbytes:
        if workspace is not None and workspace.numel() * workspace.element_size() >= nbytes:
            ws = workspace
        else:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    dev = x.device.index
    args = (*lead, xb.data_ptr(), xs, xbs, ob.data_ptr(), os_, obs, w, h, batch, levels, mode, DWT2_EXT_SYMMETRIC,
            *extra, ws.data_ptr() if ws is not None else None, nbytes, _stream(dev))
    if dev == torch.cuda.current_device():  # the library launches on the current device
        status = getattr(lib, name)(*args)
    else:
        with torch.cuda.device(x.device):
            status = getattr(lib, name)(*args)
    _lib.check(status)
    return out


def fwd(x: torch.Tensor, levels: int, mode=None, out=None, workspace=None) -> torch.Tensor:
    """Forward multi-level transform of (..., H, W); returns Mallat-packed
    coefficients of the same shape.  `workspace` (a device byte tensor of at
    least workspace_size(...) bytes) avoids a per-call allocation."""
    return _run("dwt2_fwd", x, levels, mode, out, workspace)


def inv(c: torch.Tensor, levels: int, mode=None, out=None, workspace=None) -> torch.Tensor:
    """Inverse of fwd."""
    return _run("dwt2_inv", c, levels, mode, out, workspace)


def bwd(g: torch.Tensor, levels: int, out=None, workspace=None) -> torch.Tensor:
    """Adjoint of the float forward transform: W^T g."""
    return _run("dwt2_bwd", g, levels, DWT2_F32, out, workspace)


_TUNE_DIRS = {"fwd": 0, "inv": 1, "bwd": 2, "fwd_cdf97": 3, "inv_cdf97": 4}


def tune(direction: str, x: torch.Tensor, levels: int, mode=None, out=None, workspace=None) -> torch.Tensor:
    """Tune the work-item heights of the launches of `direction` ("fwd",
    "inv", "bwd", or the CDF 9/7's "fwd_cdf97" / "inv_cdf97") on inputs
    shaped like x (see dwt2_tune): later calls of the same shapes use the
    fastest heights.  Returns the call's result."""
    if direction not in _TUNE_DIRS:
        raise ValueError("direction must be 'fwd', 'inv', 'bwd', 'fwd_cdf97' or 'inv_cdf97'")
    if direction in ("bwd", "fwd_cdf97", "inv_cdf97"):
        mode = DWT2_F32
    return _run("dwt2_tune", x, levels, mode, out, workspace, lead=(_TUNE_DIRS[direction],))


def tune_entries() -> int:
    """Launch shapes with a tuned height."""
    return int(_lib.load().dwt2_tune_entries())


def tune_clear() -> None:
    """Forget every tuned height."""
    _lib.check(_lib.load().dwt2_tune_clear())


def _image_table(srcs: Sequence[torch.Tensor], dsts: Sequence[torch.Tensor]):
    arr = (_lib.Dwt2Image * len(srcs))()
    for i, (s, d) in enumerate(zip(srcs, dsts)):
        if s.dim() != 2 or s.stride(1) != 1 or d.stride(1) != 1:
            raise ValueError(f"image {i}: need a 2-D tensor with unit column stride")
        arr[i].src, arr[i].dst = s.data_ptr(), d.data_ptr()
        arr[i].src_stride, arr[i].dst_stride = s.stride(0), d.stride(0)
        arr[i].height, arr[i].width = s.shape
    return arr


def batched_workspace_size(images: Sequence[torch.Tensor], levels: int, mode=None) -> int:
    """Bytes of device workspace dwt2_fwd_batched needs for these images."""
    if not images:
        return 0
    mode = _mode_of(images[0], mode)
    arr = _image_table(images, images)
    return int(_lib.load().dwt2_batched_workspace_size(arr, len(images), levels, mode))


# Workspaces of batched calls made without one, one per (device, shape set,
# levels, mode), at most _WS_CACHE_MAX of them: the library caches a plan
# per shape set and workspace address, so a stable workspace lets repeated
# calls replay their plan instead of building a new one.
_WS_CACHE_MAX = 4
_ws_cache: "OrderedDict[tuple, torch.Tensor]" = OrderedDict()


def _batched_workspace(images: Sequence[torch.Tensor], levels: int, mode: int, nbytes: int) -> torch.Tensor:
    dev = images[0].device
    key = (str(dev), levels, mode, tuple(tuple(t.shape) for t in images))
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        _ws_cache[key] = ws
        while len(_ws_cache) > _WS_CACHE_MAX:
            _ws_cache.popitem(last=False)
    _ws_cache.move_to_end(key)
    return ws


def synchronize() -> None:
    """Wait for the current stream and raise if a persistent launch on this
    device gave up a dependency wait (see dwt2_synchronize)."""
    _lib.check(_lib.load().dwt2_synchronize(_stream()))


def set_job_wait(max_polls: int = 0, unreachable: bool = False) -> None:
    """Poll budget of the persistent launches' dependency waits, for tests of
    the failure path (see dwt2_set_job_wait); (0, False) restores the default."""
    _lib.check(_lib.load().dwt2_set_job_wait(max_polls, 1 if unreachable else 0))


def plan_cache_size() -> int:
    """Number of batched plans the library holds (at most 16)."""
    return int(_lib.load().dwt2_plan_cache_size())


def clear_plan_cache() -> None:
    """Release every batched plan, and the workspaces kept for them here."""
    _ws_cache.clear()
    _lib.load().dwt2_clear_plan_cache()


def _batched(name: str, images: Sequence[torch.Tensor], levels: int, mode, outs, workspace) -> List[torch.Tensor]:
    lib = _lib.load()
    if not images:
        return []
    mode = _mode_of(images[0], mode)
    for t in images:
        _mode_of(t, mode)
        if not t.is_cuda:
            raise ValueError("images must be on the GPU")
    if outs is None:
        outs = [torch.empty_like(t) for t in images]
    arr = _image_table(images, outs)
    n = len(images)
    nbytes = int(lib.dwt2_batched_workspace_size(arr, n, levels, mode))
    if workspace is None:
        ws = _batched_workspace(images, levels, mode, nbytes)
    else:
        if workspace.device != images[0].device or workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError(f"workspace must be a tensor of at least {nbytes} bytes on {images[0].device}")
        ws = workspace
    with torch.cuda.device(images[0].device):
        status = getattr(lib, name)(arr, n, levels, mode, DWT2_EXT_SYMMETRIC, ws.data_ptr(), nbytes, _stream())
    _lib.check(status)
    return list(outs)


def fwd_batched(images: Sequence[torch.Tensor], levels: int, mode=None,
                outs: Sequence[torch.Tensor] | None = None,
                workspace: torch.Tensor | None = None) -> List[torch.Tensor]:
    """Forward transform of a ragged list of 2-D images in one batched call
    (see dwt2_fwd_batched).  Plans are cached per image geometry and
    workspace address; without a `workspace`, one is kept per shape set."""
    return _batched("dwt2_fwd_batched", images, levels, mode, outs, workspace)


def inv_batched(coeffs: Sequence[torch.Tensor], levels: int, mode=None,
                outs: Sequence[torch.Tensor] | None = None,
                workspace: torch.Tensor | None = None) -> List[torch.Tensor]:
    """Inverse of fwd_batched (see dwt2_inv_batched)."""
    return _batched("dwt2_inv_batched", coeffs, levels, mode, outs, workspace)


def bwd_batched(grads: Sequence[torch.Tensor], levels: int,
                outs: Sequence[torch.Tensor] | None = None,
                workspace: torch.Tensor | None = None) -> List[torch.Tensor]:
    """Adjoint of the float forward transform on a ragged list (see
    dwt2_bwd_batched)."""
    return _batched("dwt2_bwd_batched", grads, levels, DWT2_F32, outs, workspace)


class DWT2Function(torch.autograd.Function):
    """y = W x (float32, multi-level); the backward applies the hand-written
    adjoint kernel, W^T g.  Linear, so nothing is saved for backward."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, levels: int):
        ctx.levels = levels
        return fwd(x.contiguous(), levels, DWT2_F32)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return bwd(g.contiguous(), ctx.levels), None
