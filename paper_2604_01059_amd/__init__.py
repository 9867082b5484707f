"""Bit-packed GF(2) work on graph-like ZX diagrams for AMD MI355X.

The compute lives in ``libzx.so`` (HIP for gfx950, C ABI in include/zx.h);
``zx`` is its ctypes binding.  PyTorch provides device memory and streams.
"""
__all__ = ["zx"]
