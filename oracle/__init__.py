"""CPU oracle of the OECDG method (test infrastructure).

Only tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (``paper_2503_12473_amd``) never
imports it, and it imports nothing from the product except the seeded input
generators in ``paper_2503_12473_amd.inputs``.
"""
