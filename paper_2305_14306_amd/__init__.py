"""HAVSampler on MI355X: hierarchical adaptive voxel-guided point sampling (arXiv 2305.14306).

The sampler is the HIP library ``libhav.so`` (gfx950) behind the C ABI declared in
``include/hav.h``; :mod:`paper_2305_14306_amd.hav` is its thin ctypes binding. Importing
this package loads nothing; the binding loads the library on first use and raises if it
has not been built.
"""
__all__ = ["hav", "synth"]
