"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark."""
from .sky import (StackSpec, Stack, config_specs, small_spec, make_stack, make_config,
                  render_sky, cosmic_ray_hits, ENTROPY, STAR_SIGMA_PX, STAMP_HALF)

__all__ = ["StackSpec", "Stack", "config_specs", "small_spec", "make_stack", "make_config",
           "render_sky", "cosmic_ray_hits", "ENTROPY", "STAR_SIGMA_PX", "STAMP_HALF"]
