"""Seeded synthetic operands for tests and benchmarks.

This module holds no arithmetic of the multiplication method; both the CPU oracle's tests and
the GPU path's tests and benchmarks draw their operands from here.  Limbs are uint32,
little-endian, uniform over [0, 2^32), from a splitmix64 stream (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014): each 64-bit output gives two limbs,
low half first.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

SEED_BASE = 0x44B55


def splitmix64(seed, count):
    """``count`` successive splitmix64 outputs from state ``seed`` (vectorized)."""
    with np.errstate(over="ignore"):
        idx = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def limbs(seed, n):
    """n uniform uint32 limbs from the given seed."""
    if n == 0:
        return np.zeros(0, np.uint32)
    words = splitmix64(seed, (n + 1) // 2)
    return words.view(np.uint32)[:n].copy()


def operand_pair(seed, alen, blen):
    """Two independent operands drawn from one seed."""
    return limbs(seed * 2 + 1, alen), limbs(seed * 2 + 2, blen)


def all_ones(n):
    return np.full(n, 0xFFFFFFFF, np.uint32)


def power_of_two(bit, n):
    """2^bit as n limbs (bit < 32 n)."""
    a = np.zeros(n, np.uint32)
    a[bit // 32] = np.uint32(1 << (bit % 32))
    return a


def batch_lengths(seed, count, lo_bits=12, hi_bits=22, max_ratio=8.0):
    """Operand lengths of a mixed batch: the longer operand has 2^U(lo,hi) bits (rounded to
    limbs, at least one), the ratio of the lengths is U[1, max_ratio], the longer side is a or b
    by a coin flip.  Returns a list of (alen, blen)."""
    r = splitmix64(seed, 3 * count).astype(np.float64) / 2.0 ** 64
    out = []
    for i in range(count):
        bits = 2.0 ** (lo_bits + (hi_bits - lo_bits) * r[3 * i])
        big = max(1, int(round(bits / 32.0)))
        ratio = 1.0 + (max_ratio - 1.0) * r[3 * i + 1]
        small = max(1, int(round(big / ratio)))
        out.append((big, small) if r[3 * i + 2] < 0.5 else (small, big))
    return out


def mixed_batch(count=4096, seed=SEED_BASE + 2):
    """The mixed-batch workload: `count` operand pairs with batch_lengths(seed, count) (operands
    2^12..2^22 bits, length ratio U[1, 8]); pair i is operand_pair(SEED_BASE + 100000 + i, ...)."""
    return [operand_pair(SEED_BASE + 100000 + i, al, bl)
            for i, (al, bl) in enumerate(batch_lengths(seed, count))]
