"""Plain, slow CPU oracle of the DDF hot path (float64 numpy).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import anything under this package.  It shares no code
with the HIP path and imports nothing from it.
"""
