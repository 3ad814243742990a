"""CPU FP64 oracle of the STAP hot path (test infrastructure only).

Imported by the tests, the smoke check and the bench's CPU-baseline leg; never
by the GPU library, which must fail loudly rather than fall back to it.
"""
from . import metrics, stap  # noqa: F401
