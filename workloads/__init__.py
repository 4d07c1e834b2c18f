"""Seeded synthetic inputs shared by the CPU oracle's tests and the GPU path.

This package only draws random numbers and lays out geometry: voxel meshes,
true poses, hypothesis grid specifications, noise draws and occluder boxes.
It performs none of the method's arithmetic (no rendering, no unprojection,
no likelihood). Where an input needs a render (the observed image), the
caller passes the renderer in as a function, so the tests build observations
with the oracle and the benchmark builds them with the GPU library.
"""

from .scenes import (  # noqa: F401
    VOXEL,
    Camera,
    GridSpec,
    ScoreParams,
    Workload,
    assemble_observed_depth,
    box_mesh,
    camera_pan_schedule,
    camera_pan_sequence,
    make_config,
    observation_noise,
    place_occluder,
    pose_matrix,
    random_poses,
    random_scene_batch,
    rotation_grid,
    shoemake_rotations,
    smooth_trajectory,
    tracking_sequence,
    table_scene,
    look_at,
    tiny_scene,
    voxel_blob,
    voxel_mesh,
)
