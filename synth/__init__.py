"""Seeded synthetic inputs shared by the oracle-side tests and the GPU-side tests and bench.

This package holds no arithmetic of the fast-multiplication method: only a counter-based
random generator and the input distributions of the paper's experiments (uniform, normal,
small integers, badly scaled products of diagonal and random matrices).
"""
from .gen import (  # noqa: F401
    splitmix64,
    uniform01,
    normal01,
    int_uniform,
    badly_scaled,
    fig3_pair,
    make_pair,
    DISTRIBUTIONS,
)
