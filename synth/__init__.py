"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This package only draws particle clouds and region-of-interest (ROI)
workloads. It holds none of the density-estimation arithmetic, so both
sides of a parity test may import it without sharing any of the method.
ROI fields are plain strings and numbers; each side maps them to its own
representation.
"""
from .clouds import (  # noqa: F401
    Roi,
    c1_cloud,
    clumpy_cloud,
    clumpy_cloud_device,
    lattice_cloud,
    uniform_cloud,
    blob_cloud,
    paperlike_cloud,
    c1_roi,
    c2_roi,
    nested_zoom_rois,
    random_batch_rois,
    serving_trace,
    view_path,
    random_grid,
    probe_points,
    box_around,
)
