"""Counter-based random numbers for the oracle (test infrastructure only).

The paper draws nu_t ~ N(0, I) and theta uniformly over the active intervals
(Algorithm 1) but says nothing about the generator.  Both sides of the parity
check therefore implement one counter-based generator from its published
definition, each in its own code:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11).  A 128-bit counter (four 32-bit words) and a 64-bit key
  (two words) go through ten rounds.  One round multiplies word 0 and word 2 by
  the constants M0 and M1, keeps the high and low halves of both products, and
  forms the new counter (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0).  Between
  rounds the key is bumped by the Weyl constants W0, W1 (mod 2^32).
* Box-Muller (Box & Muller, 1958) in float64: two uniforms u1, u2 in (0, 1)
  give sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2).

Stream layout (shared convention with the HIP path, restated there):

* key = (seed & 0xffffffff, seed >> 32)
* counter = (j, chain, step, stream | problem << 8)
* stream 0, pair index j: the four words of one call give the normals
  nu[2j] and nu[2j + 1] (u1 from words 0-1, u2 from words 2-3).
* stream 1, j = 0: words 0-1 give the uniform u that picks theta.
* a uniform from two words (w0, w1) is (k + 0.5) * 2^-52 with
  k = (w0 >> 6) * 2^26 + (w1 >> 6), a 52-bit integer, so it is exact in
  float64 and lies strictly inside (0, 1).

Everything is vectorised with numpy uint64 arithmetic so that whole grids of
counters are evaluated at once.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
TWO_PI = 6.283185307179586  # float64 nearest to 2 pi

STREAM_NU = 0
STREAM_U = 1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on broadcastable uint arrays; returns 4 uint32 arrays."""
    x = [np.asarray(v, dtype=np.uint64) & MASK32 for v in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * x[0]          # < 2^64, exact in uint64
        p1 = M1 * x[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
    return [v.astype(np.uint32) for v in x]


def key_of(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniform52(w0, w1):
    """Two uint32 words -> float64 uniform (k + 0.5) * 2^-52, k 52-bit."""
    k = (np.asarray(w0, dtype=np.uint64) >> np.uint64(6)) * np.uint64(1 << 26) \
        + (np.asarray(w1, dtype=np.uint64) >> np.uint64(6))
    return (k.astype(np.float64) + 0.5) * 2.0 ** -52


def box_muller(u1, u2):
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = TWO_PI * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def normals(seed, step, chains, d, problem=0):
    """nu for the given step: array (len(chains), d) float64."""
    k0, k1 = key_of(seed)
    chains = np.asarray(chains, dtype=np.uint64)
    npairs = (d + 1) // 2
    j = np.arange(npairs, dtype=np.uint64)[None, :]
    c = chains[:, None]
    w = philox4x32_10(j, c, np.uint64(step), np.uint64(STREAM_NU | (problem << 8)), k0, k1)
    z0, z1 = box_muller(uniform52(w[0], w[1]), uniform52(w[2], w[3]))
    out = np.empty((len(chains), 2 * npairs), dtype=np.float64)
    out[:, 0::2] = z0
    out[:, 1::2] = z1
    return out[:, :d]


def uniforms(seed, step, chains, problem=0):
    """u that picks theta at the given step: array (len(chains),) in (0, 1)."""
    k0, k1 = key_of(seed)
    chains = np.asarray(chains, dtype=np.uint64)
    w = philox4x32_10(np.uint64(0), chains, np.uint64(step),
                      np.uint64(STREAM_U | (problem << 8)), k0, k1)
    return uniform52(w[0], w[1])
