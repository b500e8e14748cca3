"""MI355X-native separable-footprint / distance-driven CT projector engine.

The compute path lives in the C-ABI library ``libctproj.so`` (HIP kernels for gfx950);
``paper_2503_16741_amd.ctproj`` is its thin ctypes binding.  Importing this package
loads nothing: the library is opened on first use and a missing build raises.
"""
__all__ = ["synth"]
__version__ = "0.1.0"
