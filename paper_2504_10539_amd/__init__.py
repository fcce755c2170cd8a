"""MI355X-native D2Q9 Shan-Chen lattice Boltzmann step (arXiv 2504.10539 hot path).

The compute path is the HIP library built from ``csrc/`` for gfx950 and
reached through the C-ABI declared in ``include/lbm.h``; ``lbm`` is its thin
ctypes binding.  Importing the package does not load the library; importing
``paper_2504_10539_amd.lbm`` does, and fails loudly if it is not built.
"""

__all__ = ["lbm", "inputs"]
