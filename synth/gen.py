"""Counter-based seeded input generation (host side, numpy).

Every value is a pure function of (seed, stream tag, element index), so the CPU oracle and
the GPU path see bit-identical inputs, and any sub-block can be regenerated on its own.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the golden-ratio increment
0x9E3779B97F4A7C15 and each output is the state passed through the variant-13 finaliser
of MurmurHash3 (shifts 30, 27, 31 with multipliers 0xBF58476D1CE4E5B9, 0x94D049BB133111EB).

Distributions follow the workloads of the paper's experiments: Uniform(0,1) and
Uniform(-1,1) entries (section 5.1 experiments), the three distributions of the scaling
study (section 6.5), and badly scaled products D1*R*D2 with diagonal entries 10^u.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MUL1 = np.uint64(0xBF58476D1CE4E5B9)
_MUL2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = float(2.0 ** -53)

# Stream tags keep the matrices of one seed independent of each other.
TAG_A, TAG_B, TAG_G, TAG_D1, TAG_D2, TAG_D3, TAG_D4 = 1, 2, 3, 4, 5, 6, 7


def _key(seed: int, tag: int) -> np.uint64:
    # Distinct 64-bit starting states per (seed, tag); wraps modulo 2^64.
    return np.uint64((int(seed) * 0x100000001B3 + int(tag) * 0x51ED27D3A1B2C3D5) & (2**64 - 1))


def splitmix64(seed: int, tag: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs number offset .. offset+count-1 of the SplitMix64 stream keyed by (seed, tag)."""
    with np.errstate(over="ignore"):
        idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = _key(seed, tag) + idx * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _MUL1
        z = (z ^ (z >> np.uint64(27))) * _MUL2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, tag: int, shape, offset: int = 0) -> np.ndarray:
    """Uniform[0,1) doubles with 53 random mantissa bits."""
    n = int(np.prod(shape))
    z = splitmix64(seed, tag, n, offset)
    return ((z >> np.uint64(11)).astype(np.float64) * _TWO_M53).reshape(shape)


def normal01(seed: int, tag: int, shape, offset: int = 0) -> np.ndarray:
    """Standard normal doubles by the Box-Muller transform on consecutive pairs of draws."""
    n = int(np.prod(shape))
    m = (n + 1) // 2
    z = splitmix64(seed, tag, 2 * m, 2 * offset)
    u1 = ((z[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * _TWO_M53  # (0, 1]
    u2 = (z[1::2] >> np.uint64(11)).astype(np.float64) * _TWO_M53  # [0, 1)
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * m, dtype=np.float64)
    out[0::2] = rad * np.cos(2.0 * np.pi * u2)
    out[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return out[:n].reshape(shape)


def int_uniform(seed: int, tag: int, shape, lo: int = -8, hi: int = 8, offset: int = 0) -> np.ndarray:
    """Integers uniform on {lo..hi} (as doubles); modulo reduction of 64-bit draws."""
    n = int(np.prod(shape))
    z = splitmix64(seed, tag, n, offset)
    span = np.uint64(hi - lo + 1)
    return ((z % span).astype(np.int64) + lo).astype(np.float64).reshape(shape)


def _diag10(seed: int, tag: int, n: int, span: float) -> np.ndarray:
    u = uniform01(seed, tag, (n,)) * (2.0 * span) - span
    return np.power(10.0, u)


def badly_scaled(seed: int, m: int, k: int, n: int, span: float = 6.0):
    """A = D1 R1 D2 and B = D3 R2 D4 with R uniform[0,1) and diagonals 10^u, u ~ U(-span, span)
    drawn independently per row / column."""
    d1 = _diag10(seed, TAG_D1, m, span)
    d2 = _diag10(seed, TAG_D2, k, span)
    d3 = _diag10(seed, TAG_D3, k, span)
    d4 = _diag10(seed, TAG_D4, n, span)
    A = uniform01(seed, TAG_A, (m, k)) * d1[:, None] * d2[None, :]
    B = uniform01(seed, TAG_B, (k, n)) * d3[:, None] * d4[None, :]
    return A, B


def fig3_pair(seed: int, n: int, which: int):
    """The three N x N distributions of the paper's scaling experiment (section 6.5).

    Indices are 0-based: 'i < N/2' is the first half, 'j > N/2' is read as j >= N/2.
    1: all entries Uniform(0,1).
    2: A_ij ~ U(0, 1/N^2) for j >= N/2 else U(0,1); B_ij ~ U(0, 1/N^2) for i < N/2 else U(0,1).
    3: A_ij ~ U(0, N^2) for i < N/2 and j >= N/2 else U(0,1); B_ij ~ U(0, 1/N^2) for j < N/2
       else U(0,1).
    """
    A = uniform01(seed, TAG_A, (n, n))
    B = uniform01(seed, TAG_B, (n, n))
    h = n // 2
    if which == 1:
        pass
    elif which == 2:
        A[:, h:] *= 1.0 / (n * n)
        B[:h, :] *= 1.0 / (n * n)
    elif which == 3:
        A[:h, h:] *= float(n * n)
        B[:, :h] *= 1.0 / (n * n)
    else:
        raise ValueError("which must be 1, 2 or 3")
    return A, B


DISTRIBUTIONS = ("uniform01", "uniform11", "normal", "int8", "badly_scaled")

_CHUNK = 1 << 22  # elements per work item of the threaded generation (even: whole normal pairs)


def _stream(kind: str, seed: int, tag: int, shape) -> np.ndarray:
    """Element e of the stream `kind` keyed by (seed, tag), for e = 0 .. prod(shape) - 1,
    generated in chunks on a thread pool (numpy releases the GIL in its loops).  Every element
    is the same pure function of its index as in the one-piece generation, so the result is
    bitwise the same."""
    n = int(np.prod(shape))

    def piece(start: int, cnt: int) -> np.ndarray:
        if kind == "uniform01":
            return uniform01(seed, tag, (cnt,), offset=start)
        if kind == "normal":  # offsets count Box-Muller pairs
            return normal01(seed, tag, (cnt,), offset=start // 2)
        return int_uniform(seed, tag, (cnt,), offset=start)

    if n <= _CHUNK:
        return piece(0, n).reshape(shape)
    out = np.empty(n, dtype=np.float64)

    def fill(start: int) -> None:
        cnt = min(_CHUNK, n - start)
        out[start:start + cnt] = piece(start, cnt)

    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        list(ex.map(fill, range(0, n, _CHUNK)))
    return out.reshape(shape)


def make_pair(dist: str, seed: int, m: int, k: int, n: int, dtype=np.float64):
    """(A, B) of shapes (m, k) and (k, n), row-major, in the requested dtype."""
    if dist == "uniform01":
        A = _stream("uniform01", seed, TAG_A, (m, k))
        B = _stream("uniform01", seed, TAG_B, (k, n))
    elif dist == "uniform11":
        A = _stream("uniform01", seed, TAG_A, (m, k)) * 2.0 - 1.0
        B = _stream("uniform01", seed, TAG_B, (k, n)) * 2.0 - 1.0
    elif dist == "normal":
        A = _stream("normal", seed, TAG_A, (m, k))
        B = _stream("normal", seed, TAG_B, (k, n))
    elif dist == "int8":
        A = _stream("int8", seed, TAG_A, (m, k))
        B = _stream("int8", seed, TAG_B, (k, n))
    elif dist == "badly_scaled":
        A, B = badly_scaled(seed, m, k, n)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return np.ascontiguousarray(A, dtype=dtype), np.ascontiguousarray(B, dtype=dtype)
