"""The FP32 screens of the mixed form (near-pair and parked-member kernels):
the FP32 square of an FP64 offset is compared with the FP32 square of a
radius widened by a relative margin (1e-5 for the changeover, 1e-4 for the
search reach), as the bit patterns of non-negative floats.  These checks
emulate that arithmetic with numpy float32 (every operation rounded; the
kernels fuse multiply-adds, which only rounds less) on pairs placed within
a few units in 2^-24 of the boundary, and pin the two facts the kernels rely
on: no pair inside the radius is screened out, and the integer order of the
bit patterns is the float order.  Host arithmetic only."""
import numpy as np
import pytest


def fp32_square(d64):
    f = d64.astype(np.float32)
    return (f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]


def widened(r64, margin):
    return (r64 * r64 * (1.0 + margin)).astype(np.float32)


@pytest.mark.parametrize("margin", [1e-5, 1e-4])
def test_no_pair_inside_the_radius_is_screened_out(margin):
    rng = np.random.default_rng(5)
    n = 200_000
    r = 10.0 ** rng.uniform(-5, -1, n)                     # radii from 1e-5 to 0.1 au
    u = rng.normal(size=(3, n))
    u /= np.sqrt((u * u).sum(0))
    # offsets just inside the radius: |d| = r (1 - s), s from 1e-15 to 1e-7
    s = 10.0 ** rng.uniform(-15, -7, n)
    d = u * (r * (1.0 - s))
    assert ((d * d).sum(0) < r * r).all()                # inside in exact FP64
    r2f = fp32_square(d)
    bound = widened(r, margin)
    inside = r2f.view(np.int32) < bound.view(np.int32)
    assert inside.all(), int((~inside).sum())
    # and the screen is tight: pairs beyond a few margins are screened out
    d_out = u * (r * (1.0 + 3 * margin))
    assert (fp32_square(d_out).view(np.int32) >= bound.view(np.int32)).all()


def test_bit_patterns_order_as_floats():
    rng = np.random.default_rng(6)
    a = np.abs(rng.normal(size=100_000) * 10.0 ** rng.uniform(-30, 30, 100_000)).astype(np.float32)
    b = np.abs(rng.normal(size=100_000) * 10.0 ** rng.uniform(-30, 30, 100_000)).astype(np.float32)
    a[:10] = 0.0                                          # +0 orders below every positive float
    assert np.array_equal(a < b, a.view(np.int32) < b.view(np.int32))
    assert np.array_equal(a <= b, a.view(np.int32) <= b.view(np.int32))


def test_bit_patterns_order_as_doubles():
    """The FP64 candidate test of the near kernel compares squares of
    non-negative doubles the same way."""
    rng = np.random.default_rng(7)
    a = np.abs(rng.normal(size=100_000) * 10.0 ** rng.uniform(-200, 200, 100_000))
    b = np.abs(rng.normal(size=100_000) * 10.0 ** rng.uniform(-200, 200, 100_000))
    a[:10] = 0.0
    assert np.array_equal(a <= b, a.view(np.int64) <= b.view(np.int64))
