"""Counter-based random numbers for the synthetic overlap couplings.

Every coupling c_ij of the synthetic overlap matrix is a pure function of
(seed, i, j), so any block of a very large instance can be regenerated
independently and in any order.  The generator is SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) used in
counter mode: the 64-bit counter packs the seed and the two global basis-function
indices, and the SplitMix64 output function turns it into 64 random bits.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)
_S11 = np.uint64(11)

# 21 bits per function index: up to 2,097,152 basis functions per instance.
IDX_BITS = 21
MAX_INDEX = 1 << IDX_BITS


def splitmix64(counter):
    """SplitMix64 output for an array of 64-bit counters (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = np.asarray(counter, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> _S30)) * _M1
        z = (z ^ (z >> _S27)) * _M2
        return z ^ (z >> _S31)


def pair_uniform(seed, i, j):
    """U[0,1) draw for the unordered pair {i, j} (symmetric in i and j).

    The counter is (seed << 42) | (min(i,j) << 21) | max(i,j).
    """
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    ctr = (np.uint64(seed) << np.uint64(2 * IDX_BITS)) | (lo << np.uint64(IDX_BITS)) | hi
    bits = splitmix64(ctr) >> _S11                   # 53 random bits
    return bits.astype(np.float64) * (1.0 / 9007199254740992.0)
