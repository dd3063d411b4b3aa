"""Seeded synthetic inputs shared by the renderer's tests, its benchmark and the
CPU oracle.

This package draws random scenes, cameras and poses; it holds none of the
renderer's arithmetic (no projection, no colour evaluation, no blending).  Both
the HIP path and the oracle read exactly the arrays it returns.
"""
from .scenes import (  # noqa: F401
    Scene,
    Camera,
    terrain_scene,
    aerial_scene,
    partitioned_scene,
    down_pose,
    perturb_poses,
    terrain_20k_view,
    aerial_1m_1080p,
    aerial_1m_64_views,
    differentiable_200k,
    fd_subset_5k,
    partitioned_8m,
    tiny_scene,
    f32_to_bf16_bits,
    bf16_bits_to_f32,
    feature_maps,
    matching_maps,
)
