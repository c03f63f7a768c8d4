"""SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), counter form.

The paper draws the STG mode angles and phases from uniform distributions
without naming a generator.  Both the oracle and the GPU library implement
this published generator independently so a seed fixes one mode table.

Output number m (m = 1, 2, ...) of the stream seeded with s is
mix(s + m * GAMMA mod 2^64), where mix is the MurmurHash3-style finalizer
with shifts 30, 27, 31 and the two published multipliers.  A uniform double
in [0, 1) is (output >> 11) * 2^-53.
"""

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
MUL1 = 0xBF58476D1CE4E5B9
MUL2 = 0x94D049BB133111EB


def mix64(z):
    z &= MASK64
    z = ((z ^ (z >> 30)) * MUL1) & MASK64
    z = ((z ^ (z >> 27)) * MUL2) & MASK64
    return z ^ (z >> 31)


def output(seed, m):
    """The m-th output (1-based) of the stream seeded with `seed`."""
    return mix64((seed + m * GAMMA) & MASK64)


def stream(seed, count):
    """The first `count` outputs, by stepping the state as the published code does."""
    state = seed & MASK64
    out = []
    for _ in range(count):
        state = (state + GAMMA) & MASK64
        out.append(mix64(state))
    return out


def uniform(seed, m):
    """Uniform double in [0, 1) from output m (1-based)."""
    return (output(seed, m) >> 11) * 2.0 ** -53
