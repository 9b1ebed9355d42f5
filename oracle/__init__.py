"""FP64 CPU oracle of the filter chain -- test infrastructure only.

Importable only by the test suite, the smoke check and the benchmark's CPU
baseline.  The GPU library and its binding never import it.
"""
