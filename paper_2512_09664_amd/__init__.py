"""MI355X-native synthetic PIV image-pair generator (HIP kernels behind a C ABI).

The kernels live in ``libsynthpix.so`` (built from ``csrc/`` by ``build.py``);
``api`` marshals PyTorch tensors and streams into the C entry points
``synthpix_seed``, ``synthpix_advect``, ``synthpix_render_pair`` and
``synthpix_render_pair_backward``.
"""

from . import _lib  # noqa: F401
from .api import (PairBatch, Plan, advect, advect_workspace_size, render_images, advect_params, alloc_workspace, bin_views, default_tiling,  # noqa: F401
                  particle_count,
                  probe, read_status, timing_enable, timing_read,
                  mse_grad, render_pair, render_pair_backward, render_pair_backward_mse, render_pair_noalloc, render_params, seed_shape, histogram_match, flow_field, seed, seed_params, split_images, tiling, tiling_candidates,
                  workspace_size)
