"""Seeded, platform-independent random inputs.

Every random number used by the tests and the benchmark comes from the
SplitMix64 generator (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), whose output i for seed s is the mixing
function applied to s + (i + 1) * 0x9E3779B97F4A7C15.  Because the state is a
plain counter, bulk streams are generated vectorised and in parallel chunks,
and a given (seed, index) always yields the same value on every machine.

This module holds no tensor-contraction arithmetic: it only produces inputs.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_gen.so")
_lib = None


def build_native(force: bool = False) -> str:
    """Compile the bulk generator (plain C, OpenMP) next to this file."""
    src = os.path.join(_HERE, "_gen.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", src,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _native():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_native())
        i64, u64, p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        lib.wl_splitmix64.argtypes = [u64, i64, i64, p]
        lib.wl_complex_normal.argtypes = [u64, i64, i64, p]
        lib.wl_gaussian_int.argtypes = [u64, i64, i64, i64, i64, p]
        lib.wl_wide_odd.argtypes = [u64, i64, i64, p]
        lib.wl_unit_values.argtypes = [u64, i64, i64, p]
        _lib = lib
    return _lib

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def mix64_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def splitmix64_block(seed: int, start: int, n: int) -> np.ndarray:
    """Outputs start .. start+n-1 of the SplitMix64 stream with this seed."""
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & _MASK64) + idx * GAMMA
    return mix64(state)


def substream_seed(seed: int, tag: int) -> int:
    """Independent seed for a named sub-stream (tensor A, tensor B, ...)."""
    return mix64_int((seed & _MASK64) ^ mix64_int(0xD1B54A32D192ED03 * (tag + 1)))


class SplitMix64:
    """Sequential SplitMix64 stream for small draws (permutations, choices)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        return mix64_int(self.state)

    def uniform(self) -> float:
        """Uniform double in the open interval (0, 1), 53 random bits."""
        return ((self.next_u64() >> 11) + 0.5) * (1.0 / 9007199254740992.0)

    def below(self, n: int) -> int:
        """Uniform integer in [0, n) by rejection (no modulo bias)."""
        if n <= 0:
            raise ValueError("n must be positive")
        limit = (1 << 64) - ((1 << 64) % n)
        while True:
            x = self.next_u64()
            if x < limit:
                return x % n

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in the closed range [lo, hi]."""
        return lo + self.below(hi - lo + 1)

    def permutation(self, n: int) -> list[int]:
        """Fisher-Yates shuffle of range(n) (Durstenfeld's in-place form)."""
        p = list(range(n))
        for i in range(n - 1, 0, -1):
            j = self.below(i + 1)
            p[i], p[j] = p[j], p[i]
        return p

    def sample(self, n: int, k: int) -> list[int]:
        """k distinct values of range(n), in random order."""
        return self.permutation(n)[:k]

    def normal(self) -> float:
        u1, u2 = self.uniform(), self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def _uniform_from_bits(z: np.ndarray) -> np.ndarray:
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def _complex_normal_chunk(seed: int, start: int, n: int) -> np.ndarray:
    z = splitmix64_block(seed, 2 * start, 2 * n)
    u = _uniform_from_bits(z)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1)) * math.sqrt(0.5)
    t = (2.0 * math.pi) * u2
    out = np.empty(n, dtype=np.complex128)
    out.real = r * np.cos(t)
    out.imag = r * np.sin(t)
    return out


_CHUNK = 1 << 22


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def complex_normal_numpy(seed: int, n: int) -> np.ndarray:
    """n complex128 values with re, im i.i.d. N(0, 1/2) (so E|z|^2 = 1).

    Element j uses stream outputs 2j and 2j+1 through the Box-Muller
    transform; the result does not depend on chunking or thread count.
    """
    out = np.empty(n, dtype=np.complex128)
    starts = list(range(0, n, _CHUNK))

    def work(s: int) -> None:
        m = min(_CHUNK, n - s)
        out[s:s + m] = _complex_normal_chunk(seed, s, m)

    if len(starts) <= 1:
        for s in starts:
            work(s)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, starts))
    return out


def gaussian_integers_numpy(seed: int, n: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """n complex values whose re and im are uniform integers in [lo, hi].

    Sums of products of such values are exact in binary floating point as long
    as every partial sum stays below the format's integer limit, so any
    summation order gives the same bits.
    """
    z = splitmix64_block(seed, 0, 2 * n)
    span = np.uint64(hi - lo + 1)
    v = (z % span).astype(np.int64) + lo
    out = np.empty(n, dtype=np.complex128)
    out.real = v[0::2]
    out.imag = v[1::2]
    return out


def complex_normal(seed: int, n: int) -> np.ndarray:
    """n complex128 values with re, im i.i.d. N(0, 1/2) (so E|z|^2 = 1).

    Element j uses stream outputs 2j and 2j+1 through the Box-Muller
    transform (bulk C version of ``complex_normal_numpy``).
    """
    out = np.empty(n, dtype=np.complex128)
    if n:
        _native().wl_complex_normal(seed & _MASK64, 0, n, out.ctypes.data)
    return out


def gaussian_integers(seed: int, n: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """n complex values whose re and im are integers in [lo, hi].

    Sums of products of such values are exact in binary floating point as long
    as every partial sum stays below the format's integer limit, so any
    summation order gives the same bits.
    """
    out = np.empty(n, dtype=np.complex128)
    if n:
        _native().wl_gaussian_int(seed & _MASK64, 0, n, lo, hi, out.ctypes.data)
    return out


def wide_odd_integers_numpy(seed: int, n: int) -> np.ndarray:
    """n complex values whose re and im are odd integers of magnitude 257..511
    with random signs.

    Each has nine significant bits, one more than a bfloat16 holds, so its
    nearest bfloat16 differs from it by exactly 1 (a nonzero low part of a
    hi + lo bfloat16 split), while the value itself, and every product with
    a value from ``unit_values``, is exact in FP32.
    """
    z = splitmix64_block(seed, 0, 2 * n)
    mag = (257 + 2 * (z % np.uint64(128))).astype(np.int64)   # odd, 257 .. 511
    sign = np.where(((z >> np.uint64(40)) & np.uint64(1)) == 1, -1, 1)
    v = (mag * sign).astype(np.float64)
    out = np.empty(n, dtype=np.complex128)
    out.real = v[0::2]
    out.imag = v[1::2]
    return out


def unit_values_numpy(seed: int, n: int) -> np.ndarray:
    """n complex values drawn uniformly from {0, 1, -1, i, -i}: at most one
    of re, im is nonzero, so |re| + |im| <= 1."""
    z = splitmix64_block(seed, 0, n)
    table = np.array([0, 1, -1, 1j, -1j], dtype=np.complex128)
    return table[(z % np.uint64(5)).astype(np.int64)]


def wide_odd_integers(seed: int, n: int) -> np.ndarray:
    """Bulk C version of ``wide_odd_integers_numpy`` (same values)."""
    out = np.empty(n, dtype=np.complex128)
    if n:
        _native().wl_wide_odd(seed & _MASK64, 0, n, out.ctypes.data)
    return out


def unit_values(seed: int, n: int) -> np.ndarray:
    """Bulk C version of ``unit_values_numpy`` (same values)."""
    out = np.empty(n, dtype=np.complex128)
    if n:
        _native().wl_unit_values(seed & _MASK64, 0, n, out.ctypes.data)
    return out
