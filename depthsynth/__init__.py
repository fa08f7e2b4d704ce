"""Seeded synthetic depth frames for the plane-fitting hot path.

This package only renders inputs: pinhole depth images of planes and spheres,
perturbed with the Kinect depth-noise model and punched with invalid blobs.
It contains none of the plane-fitting arithmetic, so both the HIP library and
the CPU oracle can consume its frames without sharing any fitting code.
"""
from .scenes import Camera, Frame, render_scene, make_frame, camera_for, exact_plane_depth
from .configs import CONFIGS, diff_loss_inputs, frames_for, frame_for

__all__ = [
    "Camera", "Frame", "render_scene", "make_frame", "camera_for", "exact_plane_depth",
    "CONFIGS", "diff_loss_inputs", "frames_for", "frame_for",
]
