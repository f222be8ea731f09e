"""Host check of the row-transform kernels' global indexing for every supported row size.

The C2R kernel's first pass has thread t load X[k] and X[N - k] for k = t + u NT + r N / R0
(NT threads, NU rounds, first radix R0), N = n2 / 2, each load predicated to the band
columns 0..M.  At small sizes NU NT exceeds N / R0, so threads past the last butterfly form
k >= N; the predicate must then keep N - k (negative) from being loaded.  The R2C kernel's
split step forms the twiddle of column k from tw[t] and tw[k - t].  This test enumerates the
index arithmetic of those loads for n2 = 64 .. 16384 and band limits up to N - 1 and checks
every address that a predicate lets through.
"""
import pytest


def row_shape(K):
    N = 1 << K
    NT = max(64, N // 16)
    R0 = (1 << (K % 4)) if K % 4 else 16
    return N, NT, R0


@pytest.mark.parametrize("K", range(5, 14))
def test_c2r_first_pass_loads_stay_in_the_band(K):
    N, NT, R0 = row_shape(K)
    NU = (N // R0 + NT - 1) // NT
    for M in sorted({0, 1, 3, N // 4, N // 2 - 1, N - 1}):
        for t in range(NT):
            for u in range(NU):
                for r in range(R0):
                    k = t + u * NT + r * (N // R0)
                    if k <= M:                                   # X[k]
                        assert 0 <= k <= M
                    if k > 0 and k < N and N - k <= M:           # X[N - k]
                        assert 0 <= N - k <= M
                    # the split twiddle tw[k] = tw[t] tw[k - t] (table of 2N entries)
                    assert 0 <= t < 2 * N and 0 <= u * NT + r * (N // R0) < 2 * N


@pytest.mark.parametrize("K", range(5, 14))
def test_r2c_split_twiddles_stay_in_the_table(K):
    N, NT, _ = row_shape(K)
    for ncol in sorted({1, 2, N // 2, N}):
        for t in range(NT):
            for k in range(t, ncol, NT):
                assert 0 <= t < 2 * N and 0 <= k - t < 2 * N
                assert 0 <= k < ncol and 0 <= (N - k) % N < N
