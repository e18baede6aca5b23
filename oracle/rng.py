"""Counter-based random probes (oracle side).  TEST INFRASTRUCTURE ONLY.

The paper does not fix a random number generator.  Both the oracle and the
HIP library draw their probe vectors from one stateless generator, each side
implementing it separately from its published definition:

  SplitMix64 output function (Steele, Lea & Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014): for a 64-bit input x,
      z = x + 0x9E3779B97F4A7C15
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
      z = (z ^ (z >> 27)) * 0x94D049BB133111EB
      return z ^ (z >> 31)
  (all arithmetic modulo 2**64).

Counter layout: the value for (seed, tag, column c, row i) is
  mix(seed ^ (tag << 56) ^ (c << 32) ^ i),   i < 2**32, c < 2**24, tag < 128.

Rademacher:  +1 if the top bit of the hash is 0, else -1.
Gaussian:    Box-Muller on two hashes, tags `tag` and `tag | 0x80`:
             u1 = ((h1 >> 11) + 1) * 2**-53  in (0, 1]
             u2 =  (h2 >> 11)      * 2**-53  in [0, 1)
             g  = sqrt(-2 log u1) * cos(2 pi u2)

Pinned by: the published first outputs of a SplitMix64 stream seeded with 0
(tests/test_oracle_rng.py).
"""
import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Probe tags, shared by contract with the HIP side (the numbers are part of the
# counter layout, not of the method).
TAG_SLQ = 1          # Rademacher probes for SLQ / STE
TAG_PRED_Z1 = 2      # Gaussian z^(1) of the simulation algorithm
TAG_PRED_Z2 = 3      # Gaussian z^(2) of the simulation algorithm
TAG_LRAC_N = 4       # Rademacher n-part of a draw from N(0, P_LRAC)
TAG_LRAC_K = 5       # Rademacher k-part of a draw from N(0, P_LRAC)


def mix(x):
    """SplitMix64 output function applied elementwise to uint64 input."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_stream(seed, count):
    """The sequential SplitMix64 stream: state += gamma; output mix(state-gamma+gamma).

    Used only to pin `mix` against published stream outputs."""
    out = []
    state = np.uint64(seed)
    for _ in range(count):
        out.append(int(mix(np.array([state], dtype=np.uint64))[0]))
        with np.errstate(over="ignore"):
            state = state + GOLDEN_GAMMA
    return out


def counters(seed, tag, n, t, col0=0):
    """n x t array of counters for rows 0..n-1 and columns col0..col0+t-1."""
    rows = np.arange(n, dtype=np.uint64)[:, None]
    cols = np.arange(col0, col0 + t, dtype=np.uint64)[None, :]
    base = np.uint64(seed) ^ (np.uint64(tag) << np.uint64(56))
    return base ^ (cols << np.uint64(32)) ^ rows


def rademacher(seed, tag, n, t, col0=0):
    """n x t matrix of +-1 (float64), row-major [row, column]."""
    h = mix(counters(seed, tag, n, t, col0))
    return np.where((h >> np.uint64(63)) == 0, 1.0, -1.0)


def gaussian(seed, tag, n, t, col0=0):
    """n x t matrix of standard normals by Box-Muller (float64)."""
    h1 = mix(counters(seed, tag, n, t, col0))
    h2 = mix(counters(seed, tag | 0x80, n, t, col0))
    scale = 2.0 ** -53
    u1 = ((h1 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * scale
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * scale
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
