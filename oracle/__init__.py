"""The oracle: a plain FP64 CPU reference of the chaos-indicator integrator.

TEST INFRASTRUCTURE ONLY -- imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.
"""
