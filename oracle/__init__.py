"""FP64 CPU oracle for the MAC projection.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the HIP product path.
"""
