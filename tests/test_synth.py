"""The seeded input generator: the threaded chunked generation gives bitwise the same values as
generating the stream in one piece (every value is a function of its index only)."""
import numpy as np
import pytest

from synth import gen


@pytest.mark.parametrize("dist", ["uniform01", "uniform11", "normal", "int8"])
def test_chunked_generation_is_bitwise_the_one_piece_stream(dist, monkeypatch):
    m, k, n = 37, 101, 53
    whole = {
        "uniform01": lambda: (gen.uniform01(5, gen.TAG_A, (m, k)), gen.uniform01(5, gen.TAG_B, (k, n))),
        "uniform11": lambda: (gen.uniform01(5, gen.TAG_A, (m, k)) * 2.0 - 1.0,
                              gen.uniform01(5, gen.TAG_B, (k, n)) * 2.0 - 1.0),
        "normal": lambda: (gen.normal01(5, gen.TAG_A, (m, k)), gen.normal01(5, gen.TAG_B, (k, n))),
        "int8": lambda: (gen.int_uniform(5, gen.TAG_A, (m, k)), gen.int_uniform(5, gen.TAG_B, (k, n))),
    }[dist]()
    monkeypatch.setattr(gen, "_CHUNK", 256)  # many chunks, the last one partial
    A, B = gen.make_pair(dist, 5, m, k, n)
    assert np.array_equal(A, whole[0]) and np.array_equal(B, whole[1])


def test_normal_pairs_and_offsets():
    # normal01 with a pair offset continues the one-piece stream
    full = gen.normal01(9, 1, (1000,))
    assert np.array_equal(gen.normal01(9, 1, (200,), offset=150), full[300:500])
