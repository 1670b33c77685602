"""SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) as a counter-based generator, vectorised in numpy.

Stream for (seed, purpose): state_0 = (seed << 8) | purpose; output k
(k = 0, 1, ...) mixes state_0 + (k + 1) * gamma.  Purposes name the streams:
1 circuit data, 3 F2 sum-check data, 5 batch / serving draws, 6 position of
the pattern in the PM text.  (2 and 4 are the verifier's challenge streams,
which the prover and verifier implementations draw themselves.)
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

PURPOSE = {"data": 1, "gkr_chal": 2, "f2sc_data": 3, "f2sc_chal": 4,
           "mix": 5, "pm_pos": 6, "bad_entries": 7}


def splitmix64(seed: int, purpose: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+n-1 of the stream, as uint64."""
    s0 = np.uint64(((seed << 8) | purpose) & 0xFFFFFFFFFFFFFFFF)
    k = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = s0 + k * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_bits(seed: int, purpose: int, n: int, bits: int, start: int = 0) -> np.ndarray:
    """n values uniform in [0, 2^bits): the top `bits` bits of each output."""
    return splitmix64(seed, purpose, n, start) >> np.uint64(64 - bits)
