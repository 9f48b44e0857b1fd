"""Philox4x32-10 in vectorised numpy, from its published definition.

Salmon et al., SC'11, section 3.2: a 4x32-bit counter (c0, c1, c2, c3) and a
2x32-bit key (k0, k1) go through ten rounds.  One round computes the two
32x32->64 products M0*c0 and M1*c2 and sets

    (c0, c1, c2, c3) <- (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))

and between rounds the key is bumped by the Weyl constants (W0, W1).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_SH = np.uint64(32)

# Known-answer vectors published with the Random123 distribution (kat_vectors,
# "philox4x32 10"): (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0),
     (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF),
     (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=10):
    """Return the four 32-bit output words (uint32 arrays) for broadcast inputs."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = (np.array(c, dtype=np.uint64) for c in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(rounds):
        p0 = M0 * c0
        p1 = M1 * c2
        n0 = (p1 >> _SH) ^ c1 ^ k0
        n1 = p1 & _MASK
        n2 = (p0 >> _SH) ^ c3 ^ k1
        n3 = p0 & _MASK
        c0, c1, c2, c3 = n0, n1, n2, n3
        if r + 1 < rounds:
            k0 = (k0 + np.uint64(W0)) & _MASK
            k1 = (k1 + np.uint64(W1)) & _MASK
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def uniform01(word):
    """Map uint32 words to doubles in the open interval (0, 1): (w + 0.5) / 2^32."""
    return (np.asarray(word, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)
