"""Seeded synthetic profiling data: the stand-in for the hardware-counter
feature vectors of the paper's Tier 1 (Section 2) and the 64-version program
lattices of Section 3.3.

This package only draws inputs. It holds none of the suggestion method's
arithmetic (no normalisation, no regression, no ranking), so both the FP64
oracle and the GPU path may use it without sharing any of the method.
"""
from .world import World, Batch, make_batch, kernel_layout, world_for

__all__ = ["World", "Batch", "make_batch", "kernel_layout", "world_for"]
