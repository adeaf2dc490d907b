"""MI355X-native range-separated (RS) tensor pose scorer.

The work runs in librsdock.so (hand-written HIP for gfx950 behind a C ABI,
include/rsdock.h); this package holds the build script and a ctypes binding.
"""
from .rsdock import (Batch, Context, RsdError, Sinc, Tensor, build_rs_tensor, pose_order, probe_gather,  # noqa: F401
                     score_poses, score_poses_noalloc, tensor_combine, tensor_import, tensor_load)
