"""FP64 CPU oracle of the IBDL hot path: test infrastructure only.

Imported by the tests, by the package smoke check and by the benchmark's
CPU-baseline leg; never by the product path.
"""
