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
    config1,
    config2,
    config3,
    config4,
    config4_fd,
    config5,
    tiny_scene,
    f32_to_bf16_bits,
    bf16_bits_to_f32,
    feature_maps,
    matching_maps,
)
