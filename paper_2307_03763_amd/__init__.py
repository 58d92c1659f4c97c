"""MI355X-native batched Galactic-binary log-likelihood (Strub et al., arXiv:2307.03763).

The package deliberately imports nothing at load time: ``inputs`` (seeded synthetic
workloads) must stay importable without the HIP library, and the binding
(``api``) loads ``libgbx.so`` only when first used and fails loudly if it is absent.
"""

__all__ = ["api", "inputs", "drivers"]
