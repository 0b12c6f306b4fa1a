"""The count kernels' unsigned 128-bit helpers, compiled for the host and
checked against Python integers: the carry of the orbit-size scaling into
the high word, additions across 2^64 and 2^128, and the overflow flag of
leaf-group inclusion-exclusion terms."""
import ctypes
import os
import random
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("u128") / "u128_host.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared",
                           os.path.join(HERE, "native", "u128_host.cpp"), "-o", out])
    L = ctypes.CDLL(out)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.t_u128_add.argtypes = [u64p, u64p, ctypes.c_uint64, ctypes.c_uint64]
    L.t_u128_scale.argtypes = [u64p, u64p, ctypes.c_uint32]
    L.t_ie_term.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32, u64p, u64p]
    return L


def split(x):
    return ctypes.c_uint64(x & M64), ctypes.c_uint64((x >> 64) & M64)


def join(lo, hi):
    return lo.value | (hi.value << 64)


def scale(L, x, m):
    lo, hi = split(x)
    ovf = L.t_u128_scale(ctypes.byref(lo), ctypes.byref(hi), m)
    return join(lo, hi), ovf


def test_orbit_scaling_carries_into_the_high_word(lib):
    # low word alone overflows: the carry must land in the high word
    cases = [(M64, 2), (M64, 24), ((1 << 64) - 5, 4), (1 << 63, 3), (123456789 * (1 << 40), 5040),
             ((7 << 64) | M64, 720), ((1 << 127) // 24, 24)]
    for x, m in cases:
        got, ovf = scale(lib, x, m)
        assert ovf == 0 and got == x * m, (x, m)
    rng = random.Random(5)
    for _ in range(2000):
        m = rng.choice([2, 3, 4, 6, 8, 12, 24, 120, 720, 5040, rng.randrange(2, 1 << 32)])
        x = rng.getrandbits(rng.choice([63, 64, 65, 100, 120]))
        want = x * m
        got, ovf = scale(lib, x, m)
        assert ovf == (1 if want >> 128 else 0)
        assert got == want & ((1 << 128) - 1)


def test_orbit_scaling_past_128_bits_is_flagged(lib):
    for x, m in [((1 << 127), 2), ((1 << 128) - 1, 2), ((1 << 126), 5040)]:
        _, ovf = scale(lib, x, m)
        assert ovf == 1


def test_add_carries_and_flags(lib):
    rng = random.Random(6)
    for _ in range(2000):
        a = rng.getrandbits(rng.choice([10, 64, 127, 128]))
        b = rng.getrandbits(rng.choice([10, 64, 127, 128]))
        lo, hi = split(a)
        blo, bhi = split(b)
        ovf = lib.t_u128_add(ctypes.byref(lo), ctypes.byref(hi), blo.value, bhi.value)
        assert ovf == (1 if (a + b) >> 128 else 0)
        assert join(lo, hi) == (a + b) & ((1 << 128) - 1)
    lo, hi = split(M64)
    assert lib.t_u128_add(ctypes.byref(lo), ctypes.byref(hi), 1, 0) == 0 and join(lo, hi) == 1 << 64


def term(lib, coef, hs):
    arr = (ctypes.c_uint32 * max(1, len(hs)))(*hs)
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    big = lib.t_ie_term(coef, arr, len(hs), ctypes.byref(lo), ctypes.byref(hi))
    v = join(lo, hi)
    if v >> 127:
        v -= 1 << 128
    return v, big


def test_leaf_term_values_and_overflow_flag(lib):
    rng = random.Random(7)
    for _ in range(2000):
        nb = rng.randrange(1, 7)
        hs = [rng.getrandbits(rng.choice([3, 10, 16, 20])) for _ in range(nb)]
        coef = rng.choice([1, -1, 2, -6, 24, -120, 3, -15])
        want = coef
        for h in hs:
            want *= h
        v, big = term(lib, coef, hs)
        bits = abs(coef).bit_length() + sum(h.bit_length() for h in hs)
        assert big == (1 if want != 0 and bits > 120 else 0)
        if not big:
            assert v == want
    # six sets of 2^21 nodes: the product needs 126 bits -> flagged
    assert term(lib, 1, [1 << 21] * 6)[1] == 1
    assert term(lib, -120, [(1 << 20) - 1] * 5) == (-120 * ((1 << 20) - 1) ** 5, 0)
    assert term(lib, -120, [(1 << 20) - 1] * 6)[1] == 1  # 7 + 6 x 20 bits
    # any empty set makes the term 0 without a flag
    assert term(lib, 1, [1 << 31, 0, 1 << 31, 1 << 31, 1 << 31, 1 << 31]) == (0, 0)
