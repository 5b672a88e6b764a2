"""CPU oracle for the scattering self-energy: test infrastructure only.

Imported by the tests, by the smoke check and by the benchmark's CPU-baseline
leg; never by the product path.
"""
