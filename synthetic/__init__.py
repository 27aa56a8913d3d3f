"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws scenes, cameras, targets and loss weights with NumPy's
PCG64 generator.  It holds none of the rasterizer's arithmetic: no
projection, colour, sorting or blending happens here, so both the FP64
oracle and the GPU path can consume its output without sharing code.
"""
from .scenes import (Camera, Scene, LodScene, look_at, pose_camera, camera_c1, camera_c2,
                     camera_c3, cameras_c5, scene_c1, scene_c2, scene_c3,
                     scene_urban, lod_scene_c4, serve_trace_c4, target_rgb,
                     target_depth, linear_loss_weights, random_scene)

__all__ = [
    "Camera", "Scene", "LodScene", "look_at", "pose_camera", "camera_c1", "camera_c2",
    "camera_c3", "cameras_c5", "scene_c1", "scene_c2", "scene_c3",
    "scene_urban", "lod_scene_c4", "serve_trace_c4", "target_rgb",
    "target_depth", "linear_loss_weights", "random_scene",
]
