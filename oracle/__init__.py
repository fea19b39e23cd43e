"""CPU oracle for the BFV hot path.

TEST INFRASTRUCTURE ONLY.  The slow, plainly written reference the GPU
library is checked against; it shares no code with the library.  Only tests/,
the smoke check and the benchmark's CPU-baseline leg may import it.
"""
