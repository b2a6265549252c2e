"""libsparc_hip: the Chebyshev-filtered subspace iteration of the real-space
finite-difference Kohn-Sham method for periodic systems on one AMD MI355X.

    from paper_1603_04339_amd import sparc     # ctypes binding of the C ABI
    from paper_1603_04339_amd import workloads # seeded synthetic cells
"""
__all__ = ["sparc", "workloads"]
