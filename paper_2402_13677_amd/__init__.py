"""MI355X (gfx950) library for the interface-aware elliptic steps of the EBIT
phase-change method: cut fractions from edge markers, the sharp-interface heat
solve, the mass flux and the ghost-fluid pressure projection.

The compute path is ``libebit.so`` (HIP kernels behind a C ABI, declared in
include/ebit.h); ``paper_2402_13677_amd.ebit`` is a thin ctypes binding that
only marshals arguments.  Importing this package does not load the library.
"""
__all__ = ["ebit"]
