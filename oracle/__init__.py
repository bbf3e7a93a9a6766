"""CPU oracle for the encrypted logistic-regression gradient step.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the bench's cpu_baseline
leg may import this package; the product path (the HIP library and its Python
binding) never does, and shares no code with it.
"""
