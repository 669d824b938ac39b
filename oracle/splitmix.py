"""SplitMix64 buffer generator (oracle side).

The paper fills its device buffers synthetically but does not say how.  The
library fixes the fill to a counter-based generator so that any word of any
buffer can be recomputed independently on the CPU:

    word(i) = low 32 bits of SplitMix64 output number i (0-based),
              for generator state ``seed``.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; the 64-bit finaliser constants are those of the
public-domain splitmix64.c by S. Vigna): the state advances by the golden
gamma 0x9E3779B97F4A7C15, and each output is the state passed through

    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9
    z ^= z >> 27; z *= 0x94D049BB133111EB
    z ^= z >> 31

all modulo 2**64.  Output number i therefore mixes seed + (i + 1) * gamma.
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1


def mix64_int(z):
    """Finaliser on a Python int (reference form, used for tiny inputs)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def output_int(seed, i):
    """SplitMix64 output number ``i`` (0-based) for state ``seed``."""
    return mix64_int(seed + (i + 1) * GAMMA)


def word_int(seed, i):
    """32-bit buffer word ``i``: the low half of output number ``i``."""
    return output_int(seed, i) & 0xFFFFFFFF


def words(seed, start, count):
    """Words ``start .. start+count-1`` as a uint32 NumPy array.

    NumPy uint64 arithmetic wraps modulo 2**64, which is exactly the
    generator's arithmetic.
    """
    i = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + i * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return (z & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def buffer_words(seed, nbytes, chunk_words=1 << 24):
    """The whole buffer of ``nbytes`` bytes (a multiple of 4) as uint32."""
    if nbytes % 4:
        raise ValueError("buffer size must be a multiple of 4 bytes")
    n = nbytes // 4
    out = np.empty(n, dtype=np.uint32)
    for s in range(0, n, chunk_words):
        c = min(chunk_words, n - s)
        out[s:s + c] = words(seed, s, c)
    return out
