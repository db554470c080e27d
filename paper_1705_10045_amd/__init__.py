"""MI355X-native thermal multiphase lattice Boltzmann method (arXiv:1705.10045).

The compute path is the HIP library ``liblbm_mi355x.so`` built from ``csrc/``;
``paper_1705_10045_amd.lbm`` is its thin ctypes binding.  Importing the package
itself loads nothing, so the seeded input generators in ``inputs`` stay usable
without a GPU; the first call into the binding loads the library and raises if
it is missing.
"""
