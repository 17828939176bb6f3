"""Plain FP64 CPU oracle for the EP extinction-mapping hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.
"""
