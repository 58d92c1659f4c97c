"""CPU oracle of the batched Galactic-binary likelihood -- TEST INFRASTRUCTURE ONLY.

Used by tests/, by the smoke check and by the benchmark's CPU-baseline leg; the product
path (the HIP library and its binding) never imports it.
"""
