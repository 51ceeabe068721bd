"""A second Philox4x32-10, in plain Python, for the tests only.

Written from the generator's published definition (Salmon, Moraes, Dror,
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), not from the
oracle: the state is four 32-bit words, the key two; each of the ten rounds
multiplies word 0 by 0xD2511F53 and word 2 by 0xCD9E8D57 (full 64-bit
products) and recombines the halves with the other two words and the key;
the key is advanced by the Weyl increments (0x9E3779B9, 0xBB67AE85) after
every round but the last.  Used to check the oracle's stream layout against
a hand-written table (tests/golden/stream_layout_4x4.txt).
"""

MASK = 0xFFFFFFFF
MULT = (0xD2511F53, 0xCD9E8D57)
WEYL = (0x9E3779B9, 0xBB67AE85)


def block(counter, key):
    """Philox4x32-10 of a counter (4 words) under a key (2 words): 4 words."""
    x = [int(w) & MASK for w in counter]
    k = [int(w) & MASK for w in key]
    for rnd in range(10):
        prod_a = MULT[0] * x[0]
        prod_b = MULT[1] * x[2]
        x = [((prod_b >> 32) ^ x[1] ^ k[0]) & MASK,
             prod_b & MASK,
             ((prod_a >> 32) ^ x[3] ^ k[1]) & MASK,
             prod_a & MASK]
        if rnd < 9:
            k = [(k[0] + WEYL[0]) & MASK, (k[1] + WEYL[1]) & MASK]
    return x


def seeded(seed, counter):
    """The block under the key of a 64-bit seed: (low word, high word)."""
    return block(counter, (seed & MASK, (seed >> 32) & MASK))


def unit23(w):
    """(k + 1/2) 2^-23 with k the top 23 bits of w (exact in float32 and float64)."""
    return ((w >> 9) + 0.5) / 8388608.0


def unit53(w0, w1):
    """53-bit uniform in [0, 1): top 27 bits of w0, then the top 26 bits of w1."""
    return ((w0 >> 5) * 67108864 + (w1 >> 6)) / 9007199254740992.0
