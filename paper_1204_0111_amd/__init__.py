"""hsweep: moving-PML sweeping preconditioner for the 3D Helmholtz equation on MI355X.

The method is Poulson, Engquist, Li and Ying's parallel sweeping preconditioner
(panels with moving PML, multifrontal LDL^T of each panel's auxiliary problem,
the sweep applied inside GMRES(k)).  The compute path is the HIP library
libhsweep.so behind the C ABI of include/hsweep.h; `hsweep.Solver` is its
Python binding and `workloads` generates seeded synthetic inputs.
"""
