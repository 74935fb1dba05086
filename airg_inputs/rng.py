"""Counter-based SplitMix64 streams for the seeded synthetic inputs.

SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) advances a 64-bit state by the golden-gamma
0x9E3779B97F4A7C15 and returns ``mix64(state)``.  Because the state after k
steps is ``seed + k * gamma`` (mod 2^64), output k can be computed directly,
which makes it a counter-based generator: element ``i`` of stream
``(purpose, sub)`` is output number ``c + 1`` with counter
``c = purpose << 56 | sub << 40 | i``.

This module draws only the *inputs* of a solve (inflow values, permutation
keys, loss weights, batch shapes).  It holds none of the solver's arithmetic.
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

# purpose ids of the input streams (the solver's own draws use ids 1..15)
PERM = 16
G_WEST = 17
G_SOUTH = 18
LOSS_W = 19
BATCH_SIDE = 20
BATCH_THETA = 21
RHS_BATCH = 22
DEFAULT_SEED = 17517


def _mix64(z):
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def splitmix64_sequence(seed, count):
    """First ``count`` outputs of the plain sequential SplitMix64 generator."""
    k = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(np.uint64(seed & MASK64) + k * np.uint64(GAMMA))


def raw(seed, purpose, sub, n):
    """``n`` 64-bit outputs of stream (purpose, sub)."""
    if not (0 <= purpose < 256 and 0 <= sub < (1 << 16)):
        raise ValueError("purpose must fit 8 bits and sub 16 bits")
    if n >= (1 << 40):
        raise ValueError("stream too long")
    base = (purpose << 56) | (sub << 40)
    c = np.uint64(base) + np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(np.uint64(seed & MASK64) + (c + np.uint64(1)) * np.uint64(GAMMA))


def uniform(seed, purpose, sub, n):
    """U[0,1) doubles: the top 53 bits of each output times 2^-53."""
    return (raw(seed, purpose, sub, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed, purpose, sub, n):
    """N(0,1) by the Box-Muller transform of two uniform streams."""
    u = uniform(seed, purpose, sub, 2 * n)
    u1 = 1.0 - u[0::2]              # in (0, 1], so the log is finite
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
