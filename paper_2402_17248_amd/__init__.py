"""hbl: hybrid beamline tracking on one AMD MI355X (gfx950).

HIP kernels and a C ABI (libhbl.so, header include/hbl.h) for the data-parallel
hot path of a hybrid conventional + surrogate beamline simulation (Sandberg
et al., PASC '24).  ``paper_2402_17248_amd.hbl`` is the thin ctypes binding;
importing it requires the built library.
"""
__all__ = ["hbl"]
