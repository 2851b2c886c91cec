"""MI355X-native lattice-Boltzmann nanochannel solver with a Navier-slip
friction wall (Keldysh-lattice-Boltzmann hot path, arXiv 2403.15768).

The compute path is the HIP library ``liblbm.so`` behind the C ABI in
``include/lbm.h``; :mod:`paper_2403_15768_amd.lbm` is its thin ctypes binding.
Importing the package does not load the library; the binding does, and raises
if it has not been built.
"""
__all__ = ["inputs", "lbm"]
