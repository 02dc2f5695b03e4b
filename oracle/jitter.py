"""Sample-grid offsets of jittered progressive passes (test infrastructure only).

Paper, Section 2.2: while the camera does not move, further render passes raise the number of
samples per pixel and lower the image noise.  The reading implemented here (and by the HIP
library, independently): pass k of K shifts every pixel's sample grid along the ray by s ds,

    s = min(fl32(fl32(k + xi) / K), 1 - 2^-24),   xi = (z >> 48) 2^-16,

where z is output number c + 1 of a SplitMix64 stream started at `seed` for the counter
c = k 2^32 + (py W + px): z = mix(seed + (c + 1) gamma mod 2^64).  SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): gamma =
0x9E3779B97F4A7C15 and the mix is x ^= x >> 30; x *= 0xBF58476D1CE4E5B9; x ^= x >> 27;
x *= 0x94D049BB133111EB; x ^= x >> 31 (mod 2^64).  xi has 16 bits so that k + xi is exact in
float32 for K <= 256; the clamp keeps s below 1.  The running mean of the K passes tends to the
render at step / K; each pass's offsets are stratified (s K - k in [0, 1) up to rounding).
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def splitmix64_mix(z: np.ndarray) -> np.ndarray:
    """The SplitMix64 output function on uint64 arrays (arithmetic mod 2^64)."""
    z = np.asarray(z, np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def splitmix64_stream(state: int, count: int) -> list:
    """The first `count` outputs of a SplitMix64 generator whose state starts at `state`."""
    out = []
    for i in range(1, count + 1):
        x = np.uint64((state + i * GAMMA) & MASK)
        out.append(int(splitmix64_mix(np.array([x], np.uint64))[0]))
    return out


def offsets(width: int, pixels, pass_index: int, n_passes: int, seed: int) -> np.ndarray:
    """Grid offsets s (float32 values widened to float64) of `pixels` (linear indices) in pass
    `pass_index` of `n_passes`."""
    if not (1 <= n_passes <= 256 and 0 <= pass_index < n_passes):
        raise ValueError("need 0 <= pass < n_passes <= 256")
    p = np.asarray(pixels, np.uint64)
    c = (np.uint64(pass_index) << np.uint64(32)) | p
    with np.errstate(over="ignore"):
        x = np.uint64(seed & MASK) + (c + np.uint64(1)) * np.uint64(GAMMA)
    z = splitmix64_mix(x)
    xi = (z >> np.uint64(48)).astype(np.float32) * np.float32(2.0 ** -16)
    s = ((np.float32(pass_index) + xi).astype(np.float32) / np.float32(n_passes)).astype(np.float32)
    s = np.minimum(s, np.float32(1.0 - 2.0 ** -24))
    return s.astype(np.float64)
