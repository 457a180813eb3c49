"""Closed-form equilibrium shapes used as pins (FP64); they live in the
package's measurement module, shared with the comparison sweeps."""
from paper_2605_30878_amd.measure import (centre_distance, drop_on_solid, lens_area,  # noqa: F401
                                          lens_volume, plate_angle, plate_cap)
