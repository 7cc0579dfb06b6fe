"""CPU oracle for the hybrid beamline hot path -- TEST INFRASTRUCTURE ONLY.

A plain serial FP64 C implementation (``orc.c``) of everything the GPU library
computes, written independently of it from the paper (Sandberg et al.,
PASC '24) and textbook linear beam optics.  Only ``tests/``, the smoke check
and the benchmark's CPU-baseline leg may import it.  The product path never
does.
"""
from .orc import *  # noqa: F401,F403
