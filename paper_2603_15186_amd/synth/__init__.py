"""Seeded synthetic inputs shared by the renderer's tests, bench and oracle
checks.  Nothing here computes any part of the render."""
from .scenes import Scene, FloorPlan, SURFACE_DTYPE, make_random_box, make_floorplan
from .hierarchy import build_hierarchy, covariances, morton_codes
from .cameras import Camera, yaw_camera, box_camera, FreeSpace, trajectory, random_poses
from .mlpinit import mlp_init
from . import workloads

__all__ = ["Scene", "FloorPlan", "make_random_box", "make_floorplan", "build_hierarchy",
           "covariances", "morton_codes", "Camera", "yaw_camera", "box_camera",
           "FreeSpace", "trajectory", "random_poses", "mlp_init", "workloads"]
