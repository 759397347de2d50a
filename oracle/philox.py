"""Counter-based random numbers for the oracle.

The paper draws its white noise with an unspecified generator (section "Mock
generation": an independent normal variable per voxel).  Here every random
number the method needs comes from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from that
paper's definition:

* state: four 32-bit counter words (c0, c1, c2, c3) and two key words (k0, k1);
* one round: (hi0, lo0) = M0 * c0 and (hi1, lo1) = M1 * c2 as 64-bit products,
  then (c0, c1, c2, c3) <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
* between rounds the key is bumped by the Weyl constants (W0, W1);
* ten rounds.

Counter convention used throughout the method:

    key     = (seed & 0xffffffff, seed >> 32)
    counter = (idx & 0xffffffff, idx >> 32, stream, 0)

with stream 0 for the 3D box modes and stream 1 for the small-scale 1D
fields.

Uniforms: u = ((w >> 9) + 0.5) * 2**-23, in (0, 1); the 23 kept bits plus
the half make 24 significant bits, so u is exact in FP32 as well as FP64.
Normals: Box-Muller (Box & Muller 1958), z1 = r cos(2 pi u2), z2 = r sin(2 pi u2)
with r = sqrt(-2 ln u1), evaluated here in FP64.

Pins: raw words against rocRAND's Philox4x32-10 engine built and run on the
host, and the Random123 known-answer vector for the zero counter and key.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
SH32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds.  Counters are arrays (any shape) of values that
    fit in 32 bits; the key words are Python ints.  Returns four uint64
    arrays holding the 32-bit output words."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * c0          # < 2**64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> SH32, p0 & MASK32
        hi1, lo1 = p1 >> SH32, p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + W0) & 0xFFFFFFFF
        k1 = (k1 + W1) & 0xFFFFFFFF
    return c0, c1, c2, c3


def words(seed, stream, idx):
    """Philox output words for counter (idx lo, idx hi, stream, 0) and key
    (seed lo, seed hi).  idx: integer array (< 2**63).  Returns an array of
    shape idx.shape + (4,) of uint64 (32-bit values)."""
    idx = np.asarray(idx, dtype=np.uint64)
    seed = int(seed)
    out = philox4x32_10(idx & MASK32, idx >> SH32,
                        np.uint64(int(stream) & 0xFFFFFFFF), np.uint64(0),
                        seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return np.stack(out, axis=-1)


def uniform_from_word(w):
    """u = ((w >> 9) + 0.5) * 2**-23 in FP64 (exact in FP32 too)."""
    w = np.asarray(w, dtype=np.uint64)
    return ((w >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(u1, u2):
    """Two independent standard normals from two uniforms, FP64."""
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def normal_pair(seed, stream, lin):
    """The pair of normals (z1, z2) the method assigns to linear index lin.

    One Philox call serves two consecutive linear indices: index lin uses
    counter lin >> 1 and output words (2 b, 2 b + 1) with b = lin & 1.
    """
    lin = np.asarray(lin, dtype=np.uint64)
    w = words(seed, stream, lin >> np.uint64(1))
    b = (lin & np.uint64(1)).astype(np.int64)
    wa = np.take_along_axis(w, (2 * b)[..., None], axis=-1)[..., 0]
    wb = np.take_along_axis(w, (2 * b + 1)[..., None], axis=-1)[..., 0]
    return box_muller(uniform_from_word(wa), uniform_from_word(wb))
