"""Seeded synthetic CMP gathers and grid descriptions.

This package only draws inputs: grid descriptions, Ricker-wavelet hyperbolic
events, noise and trace masks.  It holds none of the transform's arithmetic, so
both the FP64 oracle and the GPU library can be fed from it without sharing any
code of the method.
"""
from .gathers import (GridDesc, CONFIGS, config_desc, ricker, ricker_gather,
                      config_gather, gaussian_sy_gather, band_limited_gather, trace_mask,
                      batch_descs, batch_gathers, random_pair, c5_batch,
                      demultiple_gather, s1_desc, s1_gather)

__all__ = ["GridDesc", "CONFIGS", "config_desc", "ricker", "ricker_gather",
           "config_gather", "gaussian_sy_gather", "band_limited_gather", "trace_mask", "batch_descs",
           "batch_gathers", "random_pair", "c5_batch", "demultiple_gather",
           "s1_desc", "s1_gather"]
