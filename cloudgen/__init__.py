"""Seeded synthetic inputs for the LSKUM sweep (geometry and connectivity only)."""
from .airfoil import (CONFIGS, KIND_INTERIOR, KIND_OUTER, KIND_WALL, Cloud, batch_sizes,
                      hilbert_order, make_airfoil_cloud, make_airfoil_clouds, naca4_thickness,
                      named_cloud)

__all__ = ["CONFIGS", "KIND_INTERIOR", "KIND_OUTER", "KIND_WALL", "Cloud", "batch_sizes",
           "hilbert_order", "make_airfoil_cloud", "make_airfoil_clouds", "naca4_thickness",
           "named_cloud"]
