"""The closure's table GELU, as the solver and training kernels evaluate it.

Each kernel looks up a linear piece in a 512-entry table and applies it;
the table (built on the host when a closure is bound) and the index
arithmetic (one float32 FMA that leaves round(32 (x + 8)) in the low
mantissa bits of x 32 + 256 + 2^23, a clamp, and a shift of the bit
pattern) are restated here from their definitions and checked against the
tanh-form GELU: within 5e-5 on [-8, 8] including every piece boundary (the
tie case), and on the outer pieces 0 below the table and x above it.  A
piece index off by one half (taking the neighbouring chord for half of
every interval) would show as an error of about 1.5e-4.
"""
import numpy as np

PER_UNIT, SEGS = 32, 512


def gelu(x):
    x = np.asarray(x, np.float64)
    return 0.5 * x * (1.0 + np.tanh(0.7978845608028654 * (x + 0.044715 * x ** 3)))


def table():
    """(slope, intercept) of piece j: the chord over the width-1/32 interval
    centred on -8 + j/32, lowered by the mean of its largest deviations."""
    h = 1.0 / PER_UNIT
    t = np.zeros((SEGS, 2), np.float32)
    for j in range(SEGS):
        x0 = -8.0 + (j - 0.5) * h
        x1 = x0 + h
        a = (gelu(x1) - gelu(x0)) / h
        b = gelu(x0) - a * x0
        xs = x0 + h * np.arange(1, 64) / 64.0
        d = gelu(xs) - (a * xs + b)
        t[j] = (a, b + 0.5 * (min(d.min(), 0.0) + max(d.max(), 0.0)))
    return t


def device_gelu(x, tab):
    """The kernels' arithmetic in float32: x 32 is exact, so adding the
    offset rounds once, as the FMA does."""
    x = np.asarray(x, np.float32)
    two23 = np.float32(2.0 ** 23)
    t = x * np.float32(PER_UNIT) + np.float32(8 * PER_UNIT + 2 ** 23)
    t = np.minimum(np.maximum(t, two23), two23 + np.float32(SEGS - 1))
    off = (t.view(np.uint32).astype(np.uint64) << 3) - (np.uint64(two23.view(np.uint32)) << 3)
    j = ((off & 0xFFFFFFFF) // 8).astype(np.int64)
    c = tab[j]
    return (c[:, 0].astype(np.float64) * x + c[:, 1]).astype(np.float32), j


def test_index_is_nearest_piece():
    tab = table()
    x = np.linspace(-8.0, 8.0, 200001, dtype=np.float32)
    _, j = device_gelu(x, tab)
    expect = np.clip(np.rint(32.0 * (x.astype(np.float64) + 8.0)), 0, SEGS - 1)
    inner = np.abs(32.0 * (x.astype(np.float64) + 8.0) % 1.0 - 0.5) > 1e-9  # ties may go either way
    assert np.array_equal(j[inner], expect[inner])


def test_table_gelu_within_5e5():
    tab = table()
    h = 1.0 / PER_UNIT
    x = np.concatenate([np.linspace(-8.0, 8.0 - 0.5 * h, 400001),
                        -8.0 + (np.arange(SEGS) + 0.5) * h]).astype(np.float32)  # every piece boundary
    y, _ = device_gelu(x, tab)
    err = np.abs(y.astype(np.float64) - gelu(x))
    assert err.max() < 5e-5, err.max()


def test_outer_pieces():
    tab = table()
    lo = np.array([-8.5, -20.0, -100.0], np.float32)
    hi = np.array([8.0, 12.0, 40.0], np.float32)
    ylo, _ = device_gelu(lo, tab)
    yhi, _ = device_gelu(hi, tab)
    assert np.all(np.abs(ylo) < 1e-3)
    assert np.all(np.abs(yhi - hi) < 1e-3 * np.maximum(1.0, hi))
