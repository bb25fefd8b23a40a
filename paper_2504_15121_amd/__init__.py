"""MI355X-native surface normals and oriented point clouds from rectified disparities.

The computation lives in hand-written HIP kernels for gfx950 behind the C ABI of
``include/snx.h`` (``libsnx.so``); this package only marshals torch device
tensors into those calls.  Entry points (same names as the C functions):

    snx_denoise, snx_affine_normals, snx_components, snx_point_cloud,
    snx_oriented_point_cloud, snx_pipeline, snx_pipeline_part (+ workspace sizes),
    snx_autotune, snx_tune_set;
    the learned filter: snx_cnn_pack, snx_cnn_denoise, snx_cnn_train_step (+ sizes);
    batch plans: Plan (snx_plan_create / run / destroy);
    adaptive supports: snx_affine_normals_star (star fill), snx_affine_normals_labels
    (window restricted to the centre's component), snx_components_creases;
    snx_components_from_edges (the labelling on an explicitly given edge graph);
    snx_compact_points (the defined points in raster order) and its
    allocation-free form snx_compact_points_noalloc.
"""
from ._lib import (snx_autotune, snx_tune_set, snx_cnn_param_count, snx_cnn_packed_bytes,
                   snx_cnn_workspace_size, snx_cnn_pack, snx_cnn_denoise, snx_cnn_train_step,
                   cnn_model, Plan, FILTER_LSQ, FILTER_CNN, POINT_DEFINED, POINT_LABELLED, SnxError, load, snx_affine_normals,
                   snx_affine_normals_labels, snx_affine_normals_star, STOP_CD, STOP_ST,
                   snx_compact_points, snx_compact_points_workspace_size, snx_components_creases,
                   snx_compact_points_noalloc, snx_components_from_edges,
                   snx_components, snx_components_workspace_size, snx_denoise,
                   snx_oriented_point_cloud, snx_pipeline, snx_pipeline_part,
                   snx_pipeline_workspace_size, snx_point_cloud, PART_FOREST, PART_POINTS)

__all__ = ["load", "snx_autotune", "snx_tune_set", "snx_cnn_param_count",
           "snx_cnn_packed_bytes", "snx_cnn_workspace_size", "snx_cnn_pack", "snx_cnn_denoise",
           "snx_cnn_train_step", "cnn_model", "Plan", "FILTER_LSQ", "FILTER_CNN", "SnxError", "POINT_DEFINED", "POINT_LABELLED", "snx_denoise",
           "snx_affine_normals", "snx_affine_normals_labels", "snx_affine_normals_star",
           "snx_compact_points", "snx_compact_points_workspace_size", "snx_components_creases",
           "snx_compact_points_noalloc", "snx_components_from_edges", "STOP_CD", "STOP_ST", "snx_components", "snx_components_workspace_size",
           "snx_point_cloud", "snx_oriented_point_cloud", "snx_pipeline", "snx_pipeline_part",
           "snx_pipeline_workspace_size"]
