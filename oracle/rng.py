"""Counter-based uniforms for the randomised-shear noise maps (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper estimates the noise of an aperture-mass map by randomising the
input many times (Sec. 1; Sec. 5.1).  The random angles are drawn from the
Philox4x64-10 generator of Salmon, Moraes, Dror & Shaw (SC'11, "Parallel
random numbers: as easy as 1, 2, 3"), so that the GPU, which must draw them
on the fly, and this oracle produce the same bits.  Definition used here:

  * key = (seed, 0), 64-bit words;
  * block counter for realisation r and block b: (b, r, 0, 0);
  * each block yields four 64-bit words; each word is split into its low
    then its high 32 bits, so block b provides the 32-bit values of pixels
    8b .. 8b+7 (pixel index = y*N + x);
  * uniform u = (v >> 8) * 2^-24 (exact in float32), angle beta = 2 pi u.

``phase_uniforms_u32`` draws these through numpy's Philox bit generator (an
independent, third-party implementation of the same algorithm).
``philox4x64_10`` is a pure-Python transcription of the published round
function; the tests pin numpy's stream and this mapping against it.
"""

import numpy as np

PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
_MASK64 = (1 << 64) - 1


def philox4x64_10(counter, key):
    """One Philox4x64-10 block, from the published definition (Python ints)."""
    c0, c1, c2, c3 = (int(v) & _MASK64 for v in counter)
    k0, k1 = (int(v) & _MASK64 for v in key)
    for _ in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & _MASK64
        hi1, lo1 = p1 >> 64, p1 & _MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + PHILOX_W0) & _MASK64
        k1 = (k1 + PHILOX_W1) & _MASK64
    return c0, c1, c2, c3


def phase_uniforms_u32(n_pix, seed, r):
    """The 32-bit Philox values of pixels 0 .. n_pix-1 of realisation r.

    numpy's Philox increments its 256-bit counter before each block, so the
    stream is started one below (r << 64), i.e. at block (0, r, 0, 0).
    """
    start = ((int(r) << 64) - 1) % (1 << 256)
    bg = np.random.Philox(key=int(seed) & _MASK64, counter=start)
    n_blocks = (n_pix + 7) // 8
    words = bg.random_raw(4 * n_blocks).astype(np.uint64)
    lo = (words & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    hi = (words >> np.uint64(32)).astype(np.uint32)
    u32 = np.empty(2 * words.size, dtype=np.uint32)
    u32[0::2] = lo
    u32[1::2] = hi
    return u32[:n_pix]


def phase_uniforms(n, seed, r):
    """Uniforms u in [0, 1) for every pixel of an n x n map, realisation r."""
    v = phase_uniforms_u32(n * n, seed, r)
    return ((v >> np.uint32(8)).astype(np.float64) * 2.0 ** -24).reshape(n, n)
