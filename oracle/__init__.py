"""CPU oracle for the EQ-hyperreduced implicit-feature-tracking ROM.

TEST INFRASTRUCTURE ONLY.  A plain, slow FP64 NumPy/SciPy implementation of
what the GPU path computes, written from the paper (Mirhoseini & Zahr,
"Accelerated solutions of convection-dominated partial differential
equations using implicit feature tracking and empirical quadrature").  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the product path never does.  It shares no code with the GPU
library: the two meet only through the seeded inputs of ``synth``.
"""
