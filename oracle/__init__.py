"""FP64 CPU oracle of the GMRES-smoothed CSG multigrid / FGMRES Helmholtz solve.

Test infrastructure only: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product path.
"""
