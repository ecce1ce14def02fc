"""The library's host moments (hk_moments_host, the values hk_build_matrix
uploads) against the oracle, integer for integer, and the entry point's
argument handling.  Host code only: runs without a GPU."""
import ctypes

import pytest

import paper_0902_0852_amd as pkg
from paper_0902_0852_amd import hk
from oracle.moments import moments

# exact factorial forms (beta = 1/m), the series with small and large p,
# the worked example's size, and the Secant workload N = 200, beta = 7/4
CASES = [
    (1, (1, 1), 64),
    (4, (1, 1), 64),
    (4, (1, 2), 64),
    (3, (5, 4), 64),
    (32, (1, 1), 512),
    (50, (3, 2), 1024),
    (37, (13, 7), 700),
    (90, (9, 5), 1200),
    (64, (1, 3), 4096),
    (60, (2, 1), 1536),
    (200, (7, 4), 2048),
]


@pytest.mark.parametrize("N,beta,K", CASES)
def test_moments_equal_oracle(N, beta, K):
    got = pkg.moments_host(N, beta, K)
    want = moments(N, beta, K)
    assert len(got) == 2 * N - 1
    bad = [n for n in range(2 * N - 1) if got[n] != want[n]]
    assert bad == []


def test_beta_is_reduced():
    assert pkg.moments_host(20, (14, 8), 512) == pkg.moments_host(20, (7, 4), 512)


def test_sizing_call_and_errors():
    L = pkg.lib()
    N = 10
    off = (ctypes.c_int64 * (2 * N))()
    beta = hk._rational((3, 2))
    assert L.hk_moments_host(N, beta, 256, None, 0, off) == 1          # sizing: HK_EINVAL + total
    total = off[2 * N - 1]
    assert total > 0
    assert all(off[i] <= off[i + 1] for i in range(2 * N - 1))
    small = (ctypes.c_uint32 * (total - 1))()
    assert L.hk_moments_host(N, beta, 256, small, total - 1, off) == 1
    words = (ctypes.c_uint32 * total)()
    assert L.hk_moments_host(N, beta, 256, words, total, off) == 0
    assert L.hk_moments_host(0, beta, 256, words, total, off) == 1     # N < 1
    assert L.hk_moments_host(N, beta, 255, words, total, off) == 1     # K odd
    assert L.hk_moments_host(N, hk._rational((0, 1)), 256, words, total, off) == 1
    assert L.hk_moments_host(N, beta, 256, words, total, None) == 1
