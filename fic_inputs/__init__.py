"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module only draws pixels.  It holds none of the encoder's arithmetic
(no pooling, no isometries, no fitting): both the oracle and the HIP path
consume the arrays it returns and nothing else from here.

The paper evaluates on medical black-and-white scans (Section I, Section VII)
that are not distributed with it, so every workload here is a synthetic stand-in
with the same structure: a flat zero background, a textured elliptical body and a
few bright filled lesions.  The recipe is spelled out in ``gen_image``.
"""
from .images import gen_image, batch_sides, BATCH_SIDES, CONFIG_SEEDS

__all__ = ["gen_image", "batch_sides", "BATCH_SIDES", "CONFIG_SEEDS"]
