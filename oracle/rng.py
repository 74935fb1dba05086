"""The solver's random draws: counter-based SplitMix64 (Steele, Lea & Flood 2014).

The paper draws a random right-hand side for each polynomial (Sec. 2.2, 2.4) and
random weights for the Luby-type CF splitting (Sec. 2.1); it fixes neither the
generator nor the distribution.  Reading: U[0,1) doubles (PETSc's default for a
random vector), element i of the stream for (purpose, level) being SplitMix64
output number c + 1 of the seed, with c = purpose << 56 | level << 40 | i.
"""
import numpy as np

PMISR = 1
POLY_RHS = 2
COARSE_RHS = 3
TRUNC_RHS = 4
CPOLY_RHS = 5   # the C-point smoother's polynomial (FC / FCF smoothing)

_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def _mix64(z):
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def uniform(seed, purpose, level, n):
    c = np.uint64((purpose << 56) | (level << 40)) + np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _mix64(np.uint64(seed) + (c + np.uint64(1)) * _GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
