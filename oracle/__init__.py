"""CPU oracle for the rational-Krylov (R-MATEX) transient of an RC power grid.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports, links or
runs anything here; only tests, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code with the GPU path: its own ordering,
sparse Cholesky (C), dense Pade matrix exponential, Arnoldi process, transient
loop, modal and dense exact solutions and trapezoidal stepping. Everything is
FP64 and written to be checked against the paper by eye, not to be fast.
"""
