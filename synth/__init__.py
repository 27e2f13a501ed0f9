"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle."""
from .surfaces import (CONFIGS, Camera, Sample, make, make_c1, make_patch, make_ortho, make_persp,
                       plane_persp, quadric_ortho, sphere_persp, tiny)

__all__ = ["CONFIGS", "Camera", "Sample", "make", "make_c1", "make_ortho", "make_patch", "make_persp",
           "plane_persp", "quadric_ortho", "sphere_persp", "tiny"]
