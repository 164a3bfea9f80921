"""MI355X-native tile-based 3D Gaussian Splatting forward renderer.

The render runs in the HIP kernels of ``librgs.so`` (C ABI in include/rgs.h);
this package is its binding.  Importing it fails if the library has not been
built: there is no CPU path.
"""
from ._binding import (FMT_FAST, FMT_PLAIN, PATHS, RGSError, Context, DeviceScene, Server, backward_scratch_size,
                       camera_struct, frame_plan, lib, new_workspace, quantize_host, render, render_backward,
                       render_debug, scene_update_plain, workspace_capacity, workspace_check, workspace_size)
from .renderer import Renderer

__all__ = ["FMT_FAST", "FMT_PLAIN", "PATHS", "RGSError", "Context", "DeviceScene", "Server", "camera_struct",
           "frame_plan", "lib", "new_workspace", "quantize_host", "render", "render_debug",
           "workspace_capacity", "workspace_check", "workspace_size", "Renderer", "backward_scratch_size",
           "render_backward", "scene_update_plain"]
