"""CPU oracle for the circuit-fitness path of arXiv:1809.11134 (QEQEA).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the HIP implementation.

``qe_oracle.c`` holds the arithmetic (fp64 fitness, float/integer encoding
updates); ``oracle.py`` is its ctypes binding; ``dense.py`` is an independent
numpy definition of the circuit unitary by Kronecker products, used to pin the
per-gate oracle.
"""
