"""MI355X-native SPOTLIGHT single-pulse search: HIP kernels behind a C-ABI
library (``libspotlight.so``) with a thin ctypes binding.

Submodules:
  ``spotlight`` -- the binding (plans, batches, search runs, ranker);
  ``workloads`` -- plan parameters and input recipes of the benchmark workloads;
  ``synth``     -- seeded synthetic filterbank blocks.
The binding is imported lazily so that the input generators work on machines
without the built library.
"""
__all__ = ["spotlight", "workloads", "synth"]
