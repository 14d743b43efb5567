"""Seeded synthetic workloads (random numbers and array layout only)."""
from .scenes import (Camera, Gaussians, KeyframePoints, MappingStream,
                     Workload, config0, mapping_stream, wall_depth,
                     config1, config2, config3_crop, frustum_gaussians,
                     identity_camera, insertion_stream, random_walk_poses,
                     room_camera, room_gaussians, sh_coefficients, tiny_scene,
                     uniform_targets, with_sh)

__all__ = ["Camera", "Gaussians", "KeyframePoints", "MappingStream",
           "Workload", "config0", "mapping_stream", "wall_depth",
           "config1", "config2", "config3_crop", "frustum_gaussians",
           "identity_camera", "insertion_stream", "random_walk_poses",
           "room_camera", "room_gaussians", "sh_coefficients", "tiny_scene",
           "uniform_targets", "with_sh"]
