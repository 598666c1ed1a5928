"""The multicore CPU comparator (pwt and dd with OpenMP) against the oracle:
bit-exact bitmaps and rank directories for several thread counts, alphabet
sizes, widths and lengths (segments shorter than a word, ragged tails),
plus out-of-range and argument errors."""
import numpy as np
import pytest

import oracle
import wtgen
from paper_1610_05994_amd import cpu_baseline as cb

CASES = [(0, 5, 1), (1, 2, 1), (7, 3, 1), (100, 1, 1), (1000, 256, 1), (4097, 20, 1), (70_001, 256, 1),
         (50_000, 1 << 12, 2), (30_000, 1 << 16, 2), (20_000, 1 << 20, 4), (3000, 1 << 24, 4)]


@pytest.mark.parametrize("algo", cb.ALGOS)
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_matches_oracle(algo, threads):
    for k, (n, sigma, w) in enumerate(CASES):
        if sigma == 1 << 24 and algo == "dd" and threads == 8:
            continue          # dd's per-thread node tables are O(threads * sigma)
        S = wtgen.uniform(n, sigma, 3100 + k).astype(wtgen.dtype_for(w))
        rc, B, R = cb.build(S, sigma, algo, threads)
        assert rc == 0
        ref = oracle.build(S, sigma)
        assert np.array_equal(B, ref.bitmaps), (algo, threads, n, sigma)
        assert np.array_equal(R, ref.ranks), (algo, threads, n, sigma)


@pytest.mark.parametrize("algo", cb.ALGOS)
def test_skewed_and_sorted_inputs(algo):
    for S, sigma in [(wtgen.zipf(200_000, 256, 1.1, 5), 256), (np.sort(wtgen.uniform(100_000, 1000, 6)), 1000),
                     (np.full(5000, 9, np.uint8), 16)]:
        rc, B, R = cb.build(S, sigma, algo, 4)
        ref = oracle.build(S, sigma)
        assert rc == 0 and np.array_equal(B, ref.bitmaps) and np.array_equal(R, ref.ranks)


@pytest.mark.parametrize("algo", cb.ALGOS)
def test_errors(algo):
    S = wtgen.uniform(1000, 100, 1).astype(np.uint8)
    S[10] = 200
    assert cb.build(S, 100, algo)[0] == 2            # symbol >= sigma
    assert cb.lib().wtc_build_dd(None, 10, 4, 1, None, None, 1) == 1
    assert cb.lib().wtc_build_pwt(S.ctypes.data, 10, 300, 1, S.ctypes.data, None, 1) == 1   # sigma > 2^8 for u8
