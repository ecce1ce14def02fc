"""Pins for the oracle's own big-integer primitives (oracle/hko.c) against
Python's independent arbitrary-precision integers."""
import random

import pytest

import oracle
from oracle.moments import rne_div


def rne_shr_ref(a, s):
    return rne_div(a, 1 << s)


def rand_int(rng, maxbits):
    b = rng.randint(0, maxbits)
    v = rng.getrandbits(b) if b else 0
    # structured values: long runs of ones / zeros exercise carries
    t = rng.random()
    if t < 0.15 and b > 0:
        v = (1 << b) - 1
    elif t < 0.25 and b > 0:
        v = 1 << (b - 1)
    return -v if rng.random() < 0.5 else v


@pytest.mark.parametrize("seed", range(6))
def test_mul_add_sub_shift(seed):
    rng = random.Random(9020852 + seed)
    for _ in range(200):
        a, b = rand_int(rng, 1200), rand_int(rng, 1200)
        s = rng.randint(0, 300)
        assert oracle.prim(0, a, b) == a * b
        assert oracle.prim(1, a, b) == a + b
        assert oracle.prim(2, a, b) == a - b
        assert oracle.prim(5, a, 0, s) == a << s
        assert oracle.prim(3, a, 0, s) == rne_shr_ref(a, s)


@pytest.mark.parametrize("seed", range(6))
def test_division(seed):
    rng = random.Random(77 + seed)
    for _ in range(200):
        a, b = rand_int(rng, 1500), rand_int(rng, 900)
        if b == 0:
            b = 1 + rng.getrandbits(40)
        assert oracle.prim(6, a, b) == abs(a) // abs(b)
        assert oracle.prim(7, a, b) == abs(a) % abs(b)
        assert oracle.prim(4, a, b) == rne_div(a, b)


def test_rounding_ties():
    # exact halves must go to the even neighbour, symmetric in sign
    for q in range(-6, 7):
        a = (2 * q + 1) << 40          # (q + 1/2) * 2^41
        want = q + 1 if (q + 1) % 2 == 0 else q
        assert oracle.prim(3, a, 0, 41) == want
        assert oracle.prim(4, 2 * q + 1, 2) == want
    assert oracle.prim(3, 0, 0, 10) == 0
    assert oracle.prim(4, 0, 7) == 0


def test_knuth_d_hard_cases():
    # qhat correction paths: divisors with top digit just above 2^31 and
    # dividends that force the add-back step
    B = 1 << 32
    cases = [
        (B ** 4 - 1, B ** 2 + 1),
        (0x7FFF800000000000_0000000000000000_00000000, 0x8000000000000000_00000001),
        (B ** 3 * 0x80000000, B * 0x80000000 + 1),
        ((B ** 5 - 1) * (B ** 2 - 1), B ** 2 - 1),
        (3 * B ** 6 + 5, B ** 3 - 3),
    ]
    for a, b in cases:
        assert oracle.prim(6, a, b) == a // b
        assert oracle.prim(7, a, b) == a % b
