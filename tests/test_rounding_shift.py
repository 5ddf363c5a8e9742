"""The rounding identity behind the kernels' integer conversions.

The fixed-point deposit weights (2^40 units per particle), the spline kernel
values and the fixed-point drift are rounded to integers on the GPU by
adding 2^52 (or 1.5 * 2^52 for signed values) to an FP64 value and reading
the low mantissa bits, instead of converting double to int64.  In
[2^52, 2^53) consecutive doubles are one apart, so the add itself rounds to
the nearest integer, ties to even, which is rint.  Checked here in IEEE FP64
on the host, over random values, exact halves and the ends of the range.
"""

import numpy as np

OFF = np.float64(2.0 ** 52)
OFF_S = np.float64(1.5 * 2.0 ** 52)


def _shift_u(t):
    return (np.asarray(t + OFF).view(np.uint64) & np.uint64((1 << 52) - 1)).astype(np.int64)


def _shift_low32(t):
    return (np.asarray(t + OFF_S).view(np.uint64) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def test_unsigned_shift_is_rint():
    rng = np.random.default_rng(11)
    t = np.concatenate([
        rng.random(200_000) * 2.0 ** rng.integers(-30, 51, 200_000),
        np.arange(0, 4096) + 0.5,                        # ties to even
        rng.integers(0, 2 ** 50, 10_000) + 0.5,
        np.array([0.0, 0.25, 0.5, 0.75, 1.5, 2.5, 2.0 ** 40, 2.0 ** 51 - 0.5, 2.0 ** 51 - 1.0]),
    ])
    assert np.all(t < 2.0 ** 51)
    assert np.array_equal(_shift_u(t), np.rint(t).astype(np.int64))


def test_signed_shift_low_bits_are_rint_modulo_2_32():
    rng = np.random.default_rng(12)
    mag = rng.random(200_000) * 2.0 ** rng.integers(-20, 51, 200_000)
    t = np.concatenate([mag * np.where(rng.random(200_000) < 0.5, -1.0, 1.0),
                        np.arange(-4096, 4096) + 0.5, np.array([-(2.0 ** 51) + 1.0, -0.5, 0.5])])
    assert np.all(np.abs(t) < 2.0 ** 51)
    want = (np.rint(t).astype(np.int64) & 0xFFFFFFFF).astype(np.uint32)
    assert np.array_equal(_shift_low32(t), want)
