"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package holds no arithmetic of the method itself: it draws primes, data
vectors, encryption randomness, vector lengths and arrival times from fixed
seeds, and converts between Python integers and little-endian 32-bit limb
arrays.  Both the HIP path and the oracle consume what it produces; neither
depends on the other.
"""
from .limbs import from_limbs, ints_from_limbs, limbs_needed, to_limbs  # noqa: F401
