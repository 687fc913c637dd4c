"""FP64 CPU reference ("oracle") for the coupled Stokes multigrid solver.

TEST INFRASTRUCTURE ONLY.  It is plain, slow and written to be checked
against the paper by eye: generic unstructured P2-P1 assembly by exact
integration, SciPy sparse matrices, the multigrid iterate of Section 3 and
the smoothers of Sections 4 and 6.  It shares no code with the HIP library.
Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import it.
"""
