"""gfx950 (MI355X) integral-equation solver for 3-D induction-log modelling with
domain-decomposition preconditioning.

The compute path is the HIP library ``libie_gfx950.so`` behind the C ABI of
``include/ie.h``; ``paper_2306_17537_amd.ie`` is its ctypes binding.  PyTorch is
used only to own device memory and streams.
"""
__all__ = ["ie"]
