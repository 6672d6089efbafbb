"""Philox counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11), written from the published description.

Philox-NxW-R applies R rounds to an N-word counter under a key of N/2 words.  A round of the
4-word variant multiplies words 0 and 2 by two fixed odd constants, keeps both halves of each
double-width product, and outputs (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
lo(M0*c0)); between rounds the key words are bumped by two Weyl constants (the golden ratio
and sqrt(3) - 1 in fixed point).

The swarm update draws its uniforms r1, r2 (Eq. 6) and its re-seeding values (mutation of
section III.B) from Philox4x32-10 with key = (seed low word, seed high word) and counter
(dimension, particle, generation, stream); a uniform in [0, 1) is (word >> 8) * 2^-24, exact
in both float32 and float64.
"""
from __future__ import annotations

import numpy as np

_CONST = {
    32: dict(M=(0xD2511F53, 0xCD9E8D57), W=(0x9E3779B9, 0xBB67AE85)),
    64: dict(M=(0xD2E7470EE14C6C93, 0xCA5A826395121157),
             W=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)),
}

STREAM_SWARM = 0      # r1 = word 0, r2 = word 1
STREAM_INIT = 1       # initial positions, word 0
STREAM_MUTATE = 2     # mutation re-seeding, word 0


def philox4(counter, key, width: int = 32, rounds: int = 10):
    """Scalar Philox4xW-R with Python integers; returns four words."""
    mask = (1 << width) - 1
    M0, M1 = _CONST[width]["M"]
    W0, W1 = _CONST[width]["W"]
    c = [int(x) & mask for x in counter]
    k0, k1 = (int(x) & mask for x in key)
    for r in range(rounds):
        if r:
            k0, k1 = (k0 + W0) & mask, (k1 + W1) & mask
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> width, p0 & mask
        hi1, lo1 = p1 >> width, p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def philox4x32_vec(c0, c1, c2, c3, key0: int, key1: int, rounds: int = 10):
    """Vectorised Philox4x32-R over arrays of counter words (broadcast); uint32 outputs."""
    m32 = np.uint64(0xFFFFFFFF)
    x = [np.asarray(v, dtype=np.uint64) & m32 for v in np.broadcast_arrays(c0, c1, c2, c3)]
    k0, k1 = np.uint64(key0 & 0xFFFFFFFF), np.uint64(key1 & 0xFFFFFFFF)
    M0, M1 = (np.uint64(v) for v in _CONST[32]["M"])
    W0, W1 = (np.uint64(v) for v in _CONST[32]["W"])
    s32 = np.uint64(32)
    for r in range(rounds):
        if r:
            k0, k1 = (k0 + W0) & m32, (k1 + W1) & m32
        p0 = M0 * x[0]
        p1 = M1 * x[2]
        x = [(p1 >> s32) ^ x[1] ^ k0, p1 & m32, (p0 >> s32) ^ x[3] ^ k1, p0 & m32]
    return [v.astype(np.uint32) for v in x]


def to_unit(word) -> np.ndarray:
    """Uniform in [0, 1) from the top 24 bits of a 32-bit word."""
    return (np.asarray(word, np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -24


def uniforms(seed: int, dims, particles, generation: int, stream: int):
    """The two uniforms (words 0 and 1) for every (particle, dim) at ``generation``.

    ``particles`` are global particle indices (frame * P + p).  Returns (u0, u1) shaped
    [len(particles), len(dims)]."""
    dims = np.asarray(dims, np.uint64)[None, :]
    parts = np.asarray(particles, np.uint64)[:, None]
    w = philox4x32_vec(dims, parts, np.uint64(generation), np.uint64(stream),
                       seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return to_unit(w[0]), to_unit(w[1])
