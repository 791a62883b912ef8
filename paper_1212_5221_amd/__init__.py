"""MI355X-native SU(3) lattice gauge fixing (Landau, Coulomb, maximally Abelian
gauge) by checkerboard overrelaxation / simulated annealing, after
Schroeck & Vogt, arXiv:1212.5221.

``paper_1212_5221_amd.gf`` is the Python binding of the C ABI in
``include/gf.h`` (``libgf.so``, HIP kernels for gfx950).
``paper_1212_5221_amd.inputs`` generates seeded synthetic configurations.
Submodules are imported lazily so that the input generator works on hosts
without a GPU.
"""
__all__ = ["gf", "inputs"]
