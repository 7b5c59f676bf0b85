"""Seeded synthetic inputs (positions, block-CSR K and S). No method arithmetic."""
from .water import (BS, BlockCSR, System, CONFIGS, build_system, make_config, streams,
                    water_cube, water_slab, trajectory, min_image, cubic_box, truncate, two_cutoffs)

__all__ = ["BS", "BlockCSR", "System", "CONFIGS", "build_system", "make_config", "streams",
           "water_cube", "water_slab", "trajectory", "min_image", "cubic_box",
           "truncate", "two_cutoffs"]
