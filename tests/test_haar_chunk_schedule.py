"""The irradiance kernel runs the Haar levels of a chunk in a different
schedule from the plain level-by-level loop (thread-local levels first, one
exchange, then the last four levels).  This emulates both schedules in
float32 -- the register schedule with the kernel's own row functions
(haar_row, haar_reg_detail in csrc/index_maps.h, compiled for the host),
the plain loop with rows from the global coefficient order -- and checks
that they write the same coefficient to the same row, bit for bit, for
every chunk length the kernel uses, and that the result is the orthonormal
Haar transform."""
import numpy as np
import pytest

from _index_maps import lib

H = np.float32(0.70710678118654752440)


def level_by_level(x, n_chunks, chunk):
    """Rows in the global order of the transform of all n_chunks chunks:
    the level with `half` details per chunk holds n_chunks * half details
    at rows n_chunks * half .. 2 n_chunks * half - 1, chunk by chunk."""
    out = {}
    x = x.copy()
    ln = x.shape[0]
    while ln > 1:
        half = ln // 2
        p, q = x[0:ln:2], x[1:ln:2]
        for i in range(half):
            out[n_chunks * half + chunk * half + i] = (p[i] - q[i]) * H
        x[:half] = (p + q) * H
        ln = half
    return out, x[0]


def register_schedule(x, n_chunks, chunk):
    L = lib()
    ch_rows = x.shape[0]
    R = ch_rows // 16
    out = {}
    sums = []
    for g in range(16):                       # one thread per (g, column)
        v = list(x[g * R:(g + 1) * R])
        half = ch_rows // 2
        n = R
        while n > 1:
            for p in range(n // 2):
                lo, hi = v[2 * p], v[2 * p + 1]
                out[L.haar_row(half, n_chunks, chunk, L.haar_reg_detail(g, n, p))] = (lo - hi) * H
                v[p] = (lo + hi) * H
            half //= 2
            n //= 2
        sums.append(v[0])
    u = sums                                  # the exchange through LDS
    half = 8
    n = 16
    while n > 1:
        for p in range(n // 2):
            lo, hi = u[2 * p], u[2 * p + 1]
            out[L.haar_row(half, n_chunks, chunk, p)] = (lo - hi) * H
            u[p] = (lo + hi) * H
        half //= 2
        n //= 2
    return out, u[0]


@pytest.mark.parametrize("n_chunks", [1, 2, 64, 1024])
def test_top_levels_follow_the_global_order(n_chunks):
    """The levels above the chunks (one chunk of n_chunks sums): detail i
    of the level with `half` details is row half + i."""
    L = lib()
    half = n_chunks // 2
    while half >= 1:
        assert [L.haar_row(half, 1, 0, i) for i in range(half)] == list(range(half, 2 * half))
        half //= 2


@pytest.mark.parametrize("ch_rows", [16, 32, 64, 128, 256])
@pytest.mark.parametrize("n_chunks,chunk", [(1, 0), (4, 3), (256, 17)])
def test_schedules_agree_bitwise(ch_rows, n_chunks, chunk):
    rng = np.random.default_rng(ch_rows * 1000 + chunk)
    x = rng.standard_normal(ch_rows).astype(np.float32)
    a, sa = level_by_level(x, n_chunks, chunk)
    b, sb = register_schedule(x, n_chunks, chunk)
    assert a.keys() == b.keys()
    assert all(np.float32(a[j]).tobytes() == np.float32(b[j]).tobytes() for j in a)
    assert np.float32(sa).tobytes() == np.float32(sb).tobytes()


@pytest.mark.parametrize("ch_rows", [16, 256])
def test_single_chunk_is_the_orthonormal_haar_transform(ch_rows):
    rng = np.random.default_rng(ch_rows)
    x = rng.standard_normal(ch_rows)
    out, s0 = register_schedule(x.astype(np.float32), 1, 0)
    coef = np.zeros(ch_rows)
    coef[0] = s0
    for j, val in out.items():
        coef[j] = val
    # orthonormal: energy is kept, and the inverse of the level recursion
    # rebuilds the input
    assert np.isclose(np.sum(coef ** 2), np.sum(x ** 2), rtol=1e-5)
    y = coef[:1].copy()
    n = 1
    while n < ch_rows:
        d = coef[n:2 * n]
        nxt = np.empty(2 * n)
        nxt[0::2] = (y + d) / np.sqrt(2.0)
        nxt[1::2] = (y - d) / np.sqrt(2.0)
        y = nxt
        n *= 2
    np.testing.assert_allclose(y, x, rtol=1e-5, atol=1e-5)
