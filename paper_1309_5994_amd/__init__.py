"""MI355X-native lattice strong-coupling Dyson solver (arXiv:1309.5994).

The compute path lives in the C-ABI library ``libscdyson.so`` (hand-written
HIP kernels for gfx950); ``paper_1309_5994_amd.scdyson`` is the thin ctypes
binding with the same entry-point names.  ``workloads`` generates the seeded
synthetic inputs.  The binding loads the library on first use and raises if it
is missing: there is no CPU fallback.
"""
__all__ = ["workloads"]
