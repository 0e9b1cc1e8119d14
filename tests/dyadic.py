"""Dyadic test inputs (small integers times powers of two) and their exact products."""
import numpy as np


def dyadic_pair(seed, m, k, n, span=6):
    """Small integers times powers of two (2^-6 .. 2^6) per row of A and per column of B: the
    scaled operands, every product and every partial sum the method forms stay exact dyadic
    numbers within FP64's 53 bits, so C is exact.  (With 2^+-12, inside factors that differ
    between the added blocks widen the sums beyond 53 bits and they round.)"""
    from synth import make_pair

    A, B = make_pair("int8", seed, m, k, n)
    rng = np.random.default_rng(seed)
    A = A * np.ldexp(1.0, rng.integers(-span, span + 1, m))[:, None]
    B = B * np.ldexp(1.0, rng.integers(-span, span + 1, n))[None, :]
    return A, B


def exact_product(A, B, shift=6):
    """A B exactly: 2^shift A and 2^shift B are integers (checked) whose int64 product stays
    below 2^53, so scaling it back by 2^(-2 shift) in FP64 is exact."""
    a = np.ldexp(A, shift)
    b = np.ldexp(B, shift)
    assert np.array_equal(a, np.rint(a)) and np.array_equal(b, np.rint(b))
    c = a.astype(np.int64) @ b.astype(np.int64)
    assert np.max(np.abs(c), initial=0) < 2 ** 53
    return np.ldexp(c.astype(np.float64), -2 * shift)
