"""MI355X-native Model Tensor Planning replan engine.

Thin ctypes binding over the C ABI in include/mtp.h (libmtp.so, hand-written
HIP for gfx950).  PyTorch only provides device memory (the workspace) and the
stream; every step of a replan runs in the library's kernels.  There is no
CPU fallback: if the library is missing, `load()` raises.
"""
from ._native import (  # noqa: F401
    MtpError, load, Plan, Batch, Server, config_struct, task_params_of, lib_path, resident_bytes,
    transient_bytes, plant_step, mix_signature, schedule_cache_lookup, schedule_cache_store, SCHEDULE_FIELDS,
    STAGE_CANDIDATES, STAGE_ROLLOUT, STAGE_TOPK, STAGE_UPDATE, STAGE_ALL,
)
