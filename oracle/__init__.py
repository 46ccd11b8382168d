"""CPU FP64 oracle for RT0/P0 Darcy flow and the BDDC method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately literal
re-statement of the paper (Sousedik, "On adaptive BDDC for the flow in
heterogeneous porous media"): sparse assembly of the mixed RT0/P0 system, a
monolithic direct solve, and the BDDC method (Algorithm "BDDC method", steps
1-3, with Algorithm "BDDC preconditioner" and Algorithm "Adaptive BDDC") built
from un-reduced local saddle-point systems.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import it; the GPU library never
does, and the two share no code.

Parity status of each function is stated in its module header.
"""
