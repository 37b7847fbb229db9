"""MI355X-native lattice Boltzmann transport pipeline (arXiv:1410.1921).

``paper_1410_1921_amd.lbm`` binds the C ABI of ``liblbm.so`` (``include/lbm.h``);
``paper_1410_1921_amd.workloads`` holds the seeded workload definitions and test
geometries.  Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["lbm", "workloads"]
