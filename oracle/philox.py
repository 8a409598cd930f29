"""Oracle: Philox4x32-10 and Box-Muller normals (test infrastructure only).

The method's random numbers (HMC momenta, Metropolis uniforms, the chi^2,
GIG and normal draws of the Gibbs blocks) come from a counter-based
generator so that any run is reproducible from (seed, chain, stream, index).
Philox4x32 with 10 rounds follows Salmon, Moraes, Dror & Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): per round,
(hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 and
c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is bumped by the Weyl
constants (W0, W1) between rounds.

Counter layout (this project's convention, shared by both sides):
  key = (seed mod 2^32, seed >> 32)
  ctr = (block, draw, (chain << 8) | stream, sub)
A block yields four uint32 words.  Uniforms are (x + 0.5) 2^-32 in float64.
Normals come from Box-Muller on word pairs (0,1) and (2,3):
  z0 = r cos(2 pi u1), z1 = r sin(2 pi u1), r = sqrt(-2 ln u0), likewise z2, z3.
Element e of a long stream uses block e >> 2, lane e & 3.

Streams: 3 HMC momenta, 4 HMC accept, 5 chi^2 (P draw), 6 GIG (Nbar draw),
7 bias draw, 8 joint-move momenta, 9 joint-move accept.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)

STREAM_MOMENTA = 3
STREAM_ACCEPT = 4
STREAM_CHI2 = 5
STREAM_GIG = 6
STREAM_BIAS = 7
STREAM_RJ_MOMENTA = 8
STREAM_RJ_ACCEPT = 9
STREAM_TAU = 10
STREAM_WARM = 11


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on arrays of 32-bit counters; returns four uint32 arrays."""
    c = [np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3)]
    k0 = np.uint64(k0) & MASK
    k1 = np.uint64(k1) & MASK
    for _ in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> S32) ^ c[1] ^ k0, p1 & MASK, (p0 >> S32) ^ c[3] ^ k1, p0 & MASK]
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return [x.astype(np.uint32) for x in c]


def words(seed, chain, stream, draw, sub, blocks):
    """uint32 words of the given Philox blocks, shape (len(blocks), 4)."""
    blocks = np.asarray(blocks, dtype=np.uint64)
    seed = int(seed)
    out = philox4x32_10(blocks, np.full_like(blocks, draw & 0xFFFFFFFF),
                        np.full_like(blocks, ((chain << 8) | stream) & 0xFFFFFFFF),
                        np.full_like(blocks, sub & 0xFFFFFFFF),
                        seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return np.stack(out, axis=-1)


def to_uniform(w):
    return (np.asarray(w, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


def box_muller(w):
    """Four normals per block from four words (shape (..., 4) -> (..., 4))."""
    u = to_uniform(w)
    r01 = np.sqrt(-2.0 * np.log(u[..., 0]))
    r23 = np.sqrt(-2.0 * np.log(u[..., 2]))
    t01 = 2.0 * np.pi * u[..., 1]
    t23 = 2.0 * np.pi * u[..., 3]
    return np.stack([r01 * np.cos(t01), r01 * np.sin(t01),
                     r23 * np.cos(t23), r23 * np.sin(t23)], axis=-1)


def normals(seed, chain, stream, draw, count, sub=0):
    """First `count` normals of one stream (element e -> block e>>2, lane e&3)."""
    nblk = (count + 3) // 4
    z = box_muller(words(seed, chain, stream, draw, sub, np.arange(nblk)))
    return z.reshape(-1)[:count]


def uniform(seed, chain, stream, draw, sub=0, block=0, lane=0):
    return float(to_uniform(words(seed, chain, stream, draw, sub, [block])[0, lane]))
