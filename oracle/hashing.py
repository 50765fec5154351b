"""Counter-based integer hash used for deterministic priorities and start
vectors: the "lowbias32" 32-bit mixer published by C. Wellons (2018, "Prospecting
for hash functions"):  x ^= x>>16; x *= 0x7feb352d; x ^= x>>15;
x *= 0x846ca68b; x ^= x>>16  (all arithmetic modulo 2^32)."""
import numpy as np


def hash32(x):
    x = np.asarray(x).astype(np.uint64) & np.uint64(0xFFFFFFFF)
    m = np.uint64(0xFFFFFFFF)
    x = x ^ (x >> np.uint64(16))
    x = (x * np.uint64(0x7FEB352D)) & m
    x = x ^ (x >> np.uint64(15))
    x = (x * np.uint64(0x846CA68B)) & m
    x = x ^ (x >> np.uint64(16))
    return x


def hash_unit(x):
    """Map ``hash32(x)`` to [-0.5, 0.5): h / 2^32 - 0.5."""
    return hash32(x).astype(np.float64) / 4294967296.0 - 0.5
