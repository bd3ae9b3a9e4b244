"""MI355X-native multiple-observer siting (arXiv 2006.16783): VIX, FINDMAX,
batched viewsheds and greedy SITE as HIP kernels behind the C ABI of
libsiting.so (include/siting.h), with a thin ctypes binding.

Importing the package loads libsiting.so and raises if it is missing; there is
no CPU fallback.
"""
from . import _lib
from ._lib import (SitingError, Schedule, OBSERVER_DTYPE, SITING_KEY_U8, SITING_KEY_F32,
                   SITING_SINK_BITMAP, SITING_SINK_COUNT, siting_abi_version, siting_device_cus,
                   siting_vix, siting_vix_stats, siting_findmax, siting_viewshed_layout, siting_viewshed_order,
                   siting_viewshed_workspace_size, siting_viewshed_default_schedule,
                   siting_viewshed_batch, siting_viewshed_r3, siting_visibility_index, siting_autotune, siting_autotune_candidates,
                   siting_greedy_workspace_size, siting_greedy, siting_greedy_noalloc,
                   SITING_GREEDY_NOALLOC_MAX_N, observers_to_device,
                   siting_cnn_param_count, siting_cnn_workspace_size, siting_cnn_forward,
                   siting_cnn_backward, siting_cnn_adam, siting_cnn_score_terrain, cnn_workspace)

__all__ = [n for n in dir() if n.startswith("siting_")] + [
    "SitingError", "Schedule", "OBSERVER_DTYPE", "observers_to_device", "cnn_workspace"]
