"""MI355X (gfx950) multi-level 2-D CDF 5/3 DWT with the non-separable lifting
scheme of Barina et al. (§3, eq. (5)): HIP kernels behind a C ABI
(include/dwt2.h), with a thin torch binding.

The HIP library is loaded on first use; `synth` (seeded inputs) needs no GPU.
"""
__all__ = ["fwd", "inv", "bwd", "fwd_batched", "inv_batched", "bwd_batched", "DWT2Function", "workspace_size",
           "batched_workspace_size", "level_sizes", "set_tiling", "set_path", "set_probe", "fwd_separable",
           "separable_workspace_size", "fwd_lds", "fwd_cdf97", "inv_cdf97", "fwd_cdf97_separable", "synchronize",
           "set_job_wait", "plan_cache_size", "clear_plan_cache", "launch_levels", "tune", "tune_entries", "tune_clear",
           "DWT2_F32", "DWT2_I32_REV"]


def __getattr__(name):
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
