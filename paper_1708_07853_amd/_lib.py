"""ctypes loader for libdwt2.so (argument marshalling only).

The library binds to the HIP runtime that is already loaded in the process;
torch is imported first so that it is torch's copy, and the loader refuses to
run if two different HIP runtimes end up mapped.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdwt2.so")

DWT2_F32 = 0
DWT2_I32_REV = 1
DWT2_EXT_SYMMETRIC = 0
STATUS = {
    0: "DWT2_OK", -1: "DWT2_ERR_ARG", -2: "DWT2_ERR_SIZE", -3: "DWT2_ERR_MODE",
    -4: "DWT2_ERR_WORKSPACE", -5: "DWT2_ERR_ALIAS", -6: "DWT2_ERR_HIP", -7: "DWT2_ERR_NOMEM",
}

# Every symbol that include/dwt2.h declares.
EXPORTS = [
    "dwt2_workspace_size", "dwt2_fwd", "dwt2_inv", "dwt2_bwd",
    "dwt2_batched_workspace_size", "dwt2_fwd_batched", "dwt2_inv_batched", "dwt2_bwd_batched",
    "dwt2_status_string", "dwt2_last_error", "dwt2_clear_plan_cache", "dwt2_set_tiling", "dwt2_set_path",
    "dwt2_set_probe", "dwt2_separable_workspace_size", "dwt2_fwd_separable", "dwt2_fwd_lds",
    "dwt2_fwd_cdf97", "dwt2_inv_cdf97", "dwt2_fwd_cdf97_separable", "dwt2_set_job_wait", "dwt2_synchronize",
    "dwt2_plan_cache_size", "dwt2_launch_levels", "dwt2_fwd_noalloc", "dwt2_tune", "dwt2_tune_entries",
    "dwt2_tune_clear",
]


class Dwt2Image(ctypes.Structure):
    _fields_ = [
        ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
        ("src_stride", ctypes.c_int64), ("dst_stride", ctypes.c_int64),
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
    ]


_lib = None


def _hip_runtimes():
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(os.path.realpath(line.split()[-1]))
    return paths


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (torch's HIP runtime must be the one we bind to)

    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_1708_07853_amd.build`")
    lib = ctypes.CDLL(path)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError(f"two HIP runtimes are mapped: {sorted(runtimes)}")
    i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    lib.dwt2_workspace_size.argtypes = [i32, i32, i32, i32, i32]
    lib.dwt2_workspace_size.restype = sz
    lib.dwt2_separable_workspace_size.argtypes = [i32, i32, i32, i32, i32]
    lib.dwt2_separable_workspace_size.restype = sz
    for name in ("dwt2_fwd", "dwt2_inv", "dwt2_bwd", "dwt2_fwd_separable", "dwt2_fwd_cdf97", "dwt2_inv_cdf97",
                 "dwt2_fwd_cdf97_separable"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, i64, i64, vp, i64, i64, i32, i32, i32, i32, i32, i32, vp, sz, vp]
        fn.restype = ctypes.c_int
    lib.dwt2_fwd_noalloc.argtypes = [vp, i64, i64, vp, i64, i64, i32, i32, i32, i32, i32, i32, vp]
    lib.dwt2_fwd_noalloc.restype = ctypes.c_int
    lib.dwt2_tune.argtypes = [i32, vp, i64, i64, vp, i64, i64, i32, i32, i32, i32, i32, i32, vp, sz, vp]
    lib.dwt2_tune.restype = ctypes.c_int
    lib.dwt2_tune_entries.argtypes = []
    lib.dwt2_tune_entries.restype = i32
    lib.dwt2_tune_clear.argtypes = []
    lib.dwt2_tune_clear.restype = ctypes.c_int
    lib.dwt2_fwd_lds.argtypes = [vp, i64, i64, vp, i64, i64, i32, i32, i32, i32, i32, i32, i32, vp, sz, vp]
    lib.dwt2_fwd_lds.restype = ctypes.c_int
    lib.dwt2_batched_workspace_size.argtypes = [ctypes.POINTER(Dwt2Image), i32, i32, i32]
    lib.dwt2_batched_workspace_size.restype = sz
    for name in ("dwt2_fwd_batched", "dwt2_inv_batched", "dwt2_bwd_batched"):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.POINTER(Dwt2Image), i32, i32, i32, i32, vp, sz, vp]
        fn.restype = ctypes.c_int
    lib.dwt2_status_string.argtypes = [ctypes.c_int]
    lib.dwt2_status_string.restype = ctypes.c_char_p
    lib.dwt2_last_error.argtypes = []
    lib.dwt2_last_error.restype = ctypes.c_char_p
    lib.dwt2_set_tiling.argtypes = [i32, i32]
    lib.dwt2_set_tiling.restype = ctypes.c_int
    lib.dwt2_set_path.argtypes = [i32]
    lib.dwt2_set_path.restype = ctypes.c_int
    lib.dwt2_set_probe.argtypes = [i32, i32, vp, vp]
    lib.dwt2_set_probe.restype = ctypes.c_int
    lib.dwt2_clear_plan_cache.argtypes = []
    lib.dwt2_clear_plan_cache.restype = None
    lib.dwt2_plan_cache_size.argtypes = []
    lib.dwt2_plan_cache_size.restype = i32
    lib.dwt2_set_job_wait.argtypes = [i32, i32]
    lib.dwt2_set_job_wait.restype = ctypes.c_int
    lib.dwt2_launch_levels.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), i32]
    lib.dwt2_launch_levels.restype = i32
    lib.dwt2_synchronize.argtypes = [vp]
    lib.dwt2_synchronize.restype = ctypes.c_int
    _lib = lib
    return lib


class Dwt2Error(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


class Dwt2ValueError(ValueError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


def check(status: int) -> None:
    if status == 0:
        return
    detail = load().dwt2_last_error().decode()
    if status in (-1, -2, -3, -4, -5):
        raise Dwt2ValueError(status, detail)
    raise Dwt2Error(status, detail)
