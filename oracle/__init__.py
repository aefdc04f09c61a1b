"""Plain FP64 CPU oracle for the timing-driven placement hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.
"""
