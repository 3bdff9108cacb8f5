"""Host-side checks of numerical identities the GPU kernels rely on.

The FMM kernels form a cell's reciprocal width 1/w, w = L 2^-l, as
2^(l - bits) times the root record's 2^bits / L (both FP64, correctly
rounded) instead of dividing: scaling by a power of two is exact, so the two
must agree bit for bit over every level, bit count and extent.
"""
import numpy as np


def test_reciprocal_width_by_power_of_two_scaling():
    rng = np.random.default_rng(12)
    L = np.concatenate([rng.uniform(1e-3, 1e7, 20000), 10.0 ** rng.uniform(-30, 30, 20000),
                        [1.0, 3.0, 0.1, 2.0 ** -40, 1e300]])
    for bits in (1, 5, 9, 16):
        S = np.ldexp(1.0, bits) / L  # the root record, correctly rounded
        for lvl in range(0, bits + 1):
            direct = 1.0 / np.ldexp(L, -lvl)
            scaled = np.ldexp(S, lvl - bits)
            assert np.array_equal(direct, scaled), (bits, lvl)


def test_non_power_of_two_scaling_is_not_exact():
    # the control: with a factor of 3 instead of a power of two, forming the
    # reciprocal from a rounded quotient does round differently for some
    # extents, so the identity above is a property of the power of two
    rng = np.random.default_rng(3)
    L = rng.uniform(1e-3, 1e7, 20000)
    assert np.any(1.0 / (L * 3.0) != (1.0 / L) / 3.0)
