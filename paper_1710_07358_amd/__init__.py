"""MI355X-native parallel reduction (arXiv 1710.07358): HIP kernels for gfx950
behind the C ABI of include/rd.h, bound here for PyTorch tensors.

The binding is imported on first use, so ``paper_1710_07358_amd.workloads``
(seeded inputs) works without the built library.
"""
_API = ("reduce", "reduce_compensated", "argreduce", "reduce_paper_design", "segmented", "scan", "rowreduce", "rowreduce_forward",
        "rowreduce_backward", "RowReduce", "Workspace", "out_dtype", "saved_bytes",
        "config_get", "config_force", "tune_load", "workspace_status", "debug_force_wait_timeout",
        "DTYPES", "OPS")


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)


__all__ = list(_API)
