"""Keyed counter-based random numbers (oracle side; test infrastructure only).

The generator is SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the n-th output from state s is
mix64(s + n*GAMMA) with GAMMA = 0x9E3779B97F4A7C15 and the finaliser

    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9
    z ^= z >> 27; z *= 0x94D049BB133111EB
    z ^= z >> 31

all modulo 2**64.  A stream is keyed by (seed, purpose, a, b, c):

    k0 = seed;  k_{t+1} = mix64(k_t + (tag_t + 1) * GAMMA)  for tag in (purpose, a, b, c)
    draw(key, i) = mix64(key + (i + 1) * GAMMA)

so draw(seed, i) with no tags is the (i+1)-th SplitMix64 output from state seed.

Derived quantities
    bucket(x, m) = ((x & 0xFFFFFFFF) * m) >> 32          in [0, m)
    sign(x)      = +1 if bit 63 of x is 0 else -1
    uniform(x)   = (x >> 11) * 2**-53                       in [0, 1)
    gauss(key,i) = sqrt(-2 ln(1 - u1)) * cos(2 pi u2),  u1 = uniform(draw(key, 2i)),
                                                         u2 = uniform(draw(key, 2i+1))
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15

# Purpose tags, one independent stream family per random object of the method.
P_TS = 1        # TensorSketch hash/sign tables h_{n,k}, sigma_{n,k}     (Sec. 3.1)
P_RRF = 2       # CountSketch of the composite range-finder sketch        (Sec. 5)
P_RRF_G = 3     # Gaussian factor of the composite sketch                 (Sec. 5)
P_LEV = 4       # uniforms of leverage-score sampling                     (Sec. 3.2)
P_INIT = 5      # Gaussian random initialisation of the factors
P_RSVD = 6      # Gaussian test matrix of the randomized SVD solve         (Alg. 5)


def _u64(x):
    return np.asarray(x, dtype=np.uint64)


def mix64(z):
    z = _u64(z)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def stream_key(seed, purpose=None, a=0, b=0, c=0):
    k = _u64([seed])
    if purpose is None:
        return k
    for tag in (purpose, a, b, c):
        k = mix64(k + _u64([GAMMA]) * _u64([tag + 1]))
    return k


def draw(key, counter):
    counter = _u64(counter)
    return mix64(_u64(key) + _u64([GAMMA]) * (counter + np.uint64(1)))


def bucket(x, m):
    return ((_u64(x) & np.uint64(0xFFFFFFFF)) * np.uint64(m)) >> np.uint64(32)


def sign(x):
    return np.where((_u64(x) >> np.uint64(63)) == 0, 1.0, -1.0)


def uniform(x):
    return (_u64(x) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def gauss(key, counter):
    counter = _u64(counter)
    u1 = uniform(draw(key, np.uint64(2) * counter))
    u2 = uniform(draw(key, np.uint64(2) * counter + np.uint64(1)))
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
