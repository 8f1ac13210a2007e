"""Seeded synthetic image generators shared by the oracle tests, the GPU tests and the bench.

This package draws pixels only. It holds none of the contrast-curve arithmetic, so the CPU oracle
and the GPU path can both take their inputs from here without sharing any of the method.
"""
from .synth import (  # noqa: F401
    CONFIGS,
    batch_images,
    blob_canvas,
    cfg1_image,
    cfg2_image,
    cfg3_image,
    random_image,
    serve_pool,
    two_level_image,
)
