"""Seeded synthetic inputs and plain-data pipeline descriptions.

This module holds no stencil, pointwise or resampling arithmetic: it only
draws random numbers and writes pipeline descriptions as plain dictionaries.
Both the FP64 oracle (``oracle/``) and the GPU path consume what it returns,
and neither of them is imported here.

Random numbers come from splitmix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the state advances by the
golden-ratio increment 0x9E3779B97F4A7C15 and each output is the state passed
through the variant-13 finaliser (shifts 30, 27, 31; multipliers
0xBF58476D1CE4E5B9 and 0x94D049BB133111EB).  A uniform float in [0, 1) is the
top 24 bits of a draw times 2^-24, so every value is exactly representable in
FP32.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1


def splitmix64_block(seed: int, start: int, n: int) -> np.ndarray:
    """Draws ``start .. start+n-1`` of the splitmix64 stream seeded by ``seed``.

    Draw i uses state ``seed + (i+1) * gamma`` (mod 2^64), so any block of
    the stream can be produced without generating what precedes it.
    """
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK) + idx * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


class SplitMix64:
    """Sequential splitmix64 stream (scalar draws for small structural choices)."""

    def __init__(self, seed: int, start: int = 0):
        self.seed = seed & _MASK
        self.pos = start

    def next_u64(self) -> int:
        self.pos += 1
        z = (self.seed + self.pos * 0x9E3779B97F4A7C15) & _MASK
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform_int(self, lo: int, hi: int) -> int:
        """Integer uniform in [lo, hi] (inclusive); modulo bias < 2^-40 here."""
        return lo + self.next_u64() % (hi - lo + 1)

    def uniform(self) -> float:
        return (self.next_u64() >> 40) * (1.0 / (1 << 24))


def uniform_image(seed: int, channels: int, height: int, width: int,
                  start: int = 0) -> np.ndarray:
    """Planar CHW float32 image, pixels uniform in [0, 1) on a 2^-24 grid."""
    n = channels * height * width
    u = splitmix64_block(seed, start, n)
    v = (u >> np.uint64(40)).astype(np.float64) * (1.0 / (1 << 24))
    return v.astype(np.float32).reshape(channels, height, width)


def dyadic_image(seed: int, channels: int, height: int, width: int,
                 denom: int = 16) -> np.ndarray:
    """Planar image with values k/denom, k in [0, denom): every partial sum of a
    normalised binomial stencil over such values is exact in FP32 (and in FP16
    for denom <= 16), so results do not depend on summation order."""
    u = splitmix64_block(seed, 0, channels * height * width)
    k = (u >> np.uint64(40)) % np.uint64(denom)
    return (k.astype(np.float64) / denom).astype(np.float32).reshape(
        channels, height, width)


def integer_image(seed: int, channels: int, height: int, width: int,
                  lo: int, hi: int) -> np.ndarray:
    """Planar CHW int64 image with values in [lo, hi] (the top 32 bits of
    each draw reduced modulo hi - lo + 1; the caller casts to the storage
    type)."""
    u = splitmix64_block(seed, 0, channels * height * width)
    k = (u >> np.uint64(32)) % np.uint64(hi - lo + 1)
    return (k.astype(np.int64) + lo).reshape(channels, height, width)


def white_squares(img: np.ndarray, seed: int, count: int = 200,
                  side_lo: int = 8, side_hi: int = 128) -> np.ndarray:
    """Paints ``count`` axis-aligned squares of value 1.0 into every channel.

    Sides are uniform in [side_lo, side_hi] and top-left corners uniform over
    the positions that keep the square inside the image; squares are painted
    in draw order.  The draws continue the image's stream after its pixels.
    """
    c, h, w = img.shape
    rng = SplitMix64(seed, start=c * h * w)
    out = img.copy()
    for _ in range(count):
        side = min(rng.uniform_int(side_lo, side_hi), h, w)
        y = rng.uniform_int(0, h - side)
        x = rng.uniform_int(0, w - side)
        out[:, y:y + side, x:x + side] = 1.0
    return out


def ramp_mask(height: int, width: int) -> np.ndarray:
    """Single-channel blend mask: clamp((x - 0.4 W) / (0.2 W), 0, 1), as FP32."""
    x = np.arange(width, dtype=np.float64)
    row = np.clip((x - 0.4 * width) / (0.2 * width), 0.0, 1.0)
    return np.broadcast_to(row, (1, height, width)).astype(np.float32).copy()


def batch_sizes(seed: int, count: int, lo: int = 512, hi: int = 4096):
    """``count`` (width, height) pairs, each side uniform in [lo, hi]."""
    rng = SplitMix64(seed)
    return [(rng.uniform_int(lo, hi), rng.uniform_int(lo, hi)) for _ in range(count)]


from . import pipelines  # noqa: E402,F401  (plain-data pipeline descriptions)
