"""Sanitizer builds of the CPU code: the oracle's C source and the library's
host arithmetic (the correctly rounded moments and the multiprecision helpers
of the drivers), each compiled with its own harness under AddressSanitizer and
UndefinedBehaviorSanitizer (any report ends the run with a non-zero status),
run on small jobs that reach their branches, and compared with the ordinary
oracle and with Python integers."""
import os
import random
import shutil
import subprocess
from fractions import Fraction

import pytest

import oracle
from oracle.moments import moments

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


@pytest.fixture(scope="module")
def bins(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    hko = str(d / "hko_san")
    host = str(d / "host_san")
    subprocess.check_call(["gcc", "-std=c99", "-fopenmp"] + SAN +
                          ["-o", hko, os.path.join(HERE, "san", "hko_main.c")])
    subprocess.check_call(["g++", "-std=c++17", "-pthread"] + SAN +
                          ["-o", host, os.path.join(HERE, "san", "host_main.cpp")])
    return hko, host


def run(cmd, text_in=""):
    p = subprocess.run(cmd, input=text_in, capture_output=True, text=True, env=ENV, timeout=600)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    return p.stdout


def hx(v):
    return ("-" if v < 0 else "") + format(abs(v), "x")


def unhx(s):
    return -int(s[1:], 16) if s.startswith("-") else int(s, 16)


@pytest.mark.parametrize("N,beta,K,xn,g", [(9, (7, 4), 320, 3, 64), (12, (1, 2), 512, -5, 0),
                                           (6, (1, 1), 128, 1 << 200, 0)])
def test_oracle_factor_and_solve_under_sanitizers(bins, N, beta, K, xn, g):
    X = moments(N, beta, K)
    xf = xn << (K - K // 2)
    rng = random.Random(9020852 + N)
    b = [rng.randrange(-(1 << K), 1 << K) for _ in range(N)]
    job = ["factor", "%d %d %d" % (N, K, g)] + [hx(v) for v in X] + [hx(xf)] + [hx(v) for v in b]
    out = run([bins[0]], "\n".join(job) + "\n")
    got = {}
    for line in out.split("\n"):
        if line:
            k, i, j, *v = line.split()
            got[(k, int(i), int(j) if v else None)] = unhx(v[0] if v else j)
    of = oracle.factor_from_moments(X, N, K, xf)
    for pc in range(N):
        for r, v in zip(range(pc, N), of.column_C(pc)):
            assert got[("C", pc, r)] == v
    for pc in range(N - 1):
        for r, v in zip(range(pc + 1, N), of.column_L(pc)):
            assert got[("L", pc, r)] == v
    try:
        y = oracle.solve(of, b, 3, g)
    except ValueError:      # a zero pivot: no solve
        y = None
    if y is None:
        assert not any(k[0] == "Y" for k in got)
    else:
        assert [got[("Y", i, None)] for i in range(N)] == y


def test_oracle_primitives_under_sanitizers(bins):
    rng = random.Random(7)
    lines, cases = ["prim"], []
    for _ in range(400):
        op = rng.randrange(8)
        a = rng.choice([rng.getrandbits(rng.randrange(1, 900)), (1 << rng.randrange(1, 600)) - 1, 0])
        b = rng.choice([rng.getrandbits(rng.randrange(1, 500)) | 1, (1 << rng.randrange(1, 300)) + 1])
        a, b = a * rng.choice([1, -1]), b * rng.choice([1, -1])
        s = rng.randrange(0, 700)
        lines += ["%d %d" % (op, s), hx(a), hx(b)]
        cases.append((op, a, b, s))
    out = run([bins[0]], "\n".join(lines) + "\n").split()
    assert len(out) == len(cases)
    for (op, a, b, s), r in zip(cases, out):
        want = {0: lambda: a * b, 1: lambda: a + b, 2: lambda: a - b, 3: lambda: round(Fraction(a, 1 << s)),
                4: lambda: round(Fraction(a, b)), 5: lambda: a << s, 6: lambda: abs(a) // abs(b),
                7: lambda: abs(a) % abs(b)}[op]()
        assert unhx(r) == want, (op, a, b, s)


@pytest.mark.parametrize("N,beta,K", [(8, (7, 4), 256), (12, (1, 3), 512), (10, (5, 2), 384), (6, (3, 8), 192)])
def test_host_moments_under_sanitizers(bins, N, beta, K):
    out = run([bins[1], "moments", str(N), str(beta[0]), str(beta[1]), str(K)]).split()
    assert [unhx(v) for v in out] == moments(N, beta, K)


def test_host_multiprecision_under_sanitizers(bins):
    out = run([bins[1], "mp", "11", "600"])
    n = 0
    for line in out.split("\n"):
        if not line:
            continue
        f = line.split()
        a, b, q, r, p, s_, rd, fd, cd = (unhx(v) for v in f[:9])
        sh, rs, dec = int(f[9]), unhx(f[10]), int(f[11])
        A, B = abs(a), abs(b)
        assert (q, r) == (A // B, A % B)
        assert p == a * b and s_ == a + b
        assert rd == round(Fraction(a, B)) and fd == a // B and cd == -((-a) // B)
        assert rs == round(Fraction(a, 1 << sh)) and dec == a
        n += 1
    assert n == 600
