"""MI355X (gfx950) differentiable sparse-voxel tile rasterizer: the hot path of
the LiteVoxel training loop (arXiv 2511.02510), behind the C-ABI declared in
include/litevoxel.h.  The HIP library must be built (there is no fallback)."""
from .raster import (  # noqa: F401
    Context, Voxels, Frame, Renderer, RasterizeFn, LiteVoxelError, rasterize, settings,
    query_sizes, forward, backward, check_overflow, pass_stats, export_bins, lf_weight_workspace_size,
    lf_weight, lf_weight_noalloc, l1_grad, gamma_schedule, quantile_workspace_size, depth_quantile, depth_bins,
    depth_cutoff, graph_begin, graph_end, graph_launch, graph_reset, autotune, tune_key, set_timing,
    read_timings,
    guard_params, guard_workspace_size, prune_guard, split_params, split_workspace_size,
    footprint_range, subdivide_select, subdivide_apply,
    forward_aux, backward_aux, aux_loss, RasterizeAuxFn, rasterize_aux,
)
