"""Host-side check of the padded LDS line layout the frame FFTs use: element
n of a line sits at n + n/32, and the Stockham stages address it as a
per-butterfly base plus compile-time steps wherever the stride allows.  The
stage plan (radix 8, then 4 or 2, one radix-3 stage first for 3 * 2^a; a
final radix-16 stage in place of two radix-4 ones where a line has N / 16
threads) and the conditions below restate the kernels' compile-time rules;
the tests check that every base-plus-step address equals the element-wise
one and that the stage sequence computes the DFT."""

import numpy as np
import pytest


def ilog2(n):
    return 0 if n <= 1 else 1 + ilog2(n // 2)


def has3(n):
    return 1 if n % 3 == 0 else 0


def log2m(n):
    return ilog2(n // 3 if has3(n) else n)


def nstages(n):
    L = log2m(n)
    if L % 3 == 0:
        return has3(n) + L // 3
    if L % 3 == 2:
        return has3(n) + L // 3 + 1
    return has3(n) + (L // 3 + 1 if L >= 3 else 1)


def radix_pow2(L, t):
    if L % 3 == 0:
        return 8
    if L % 3 == 2:
        return 8 if t < L // 3 else 4
    return (8 if t < L // 3 - 1 else 4) if L >= 3 else 2


def radix(n, s):
    return 3 if (has3(n) and s == 0) else radix_pow2(log2m(n), s - has3(n))


def pstride(n, s):
    return 1 if s == 0 else pstride(n, s - 1) * radix(n, s - 1)


def fpi(n):
    return n + (n >> 5)


def pstep(d):
    return d + d // 32


@pytest.mark.parametrize("N", [64, 128, 192, 256, 384, 512, 1024, 2048])
def test_padded_stage_addresses(N):
    prod = 1
    for s in range(nstages(N)):
        R, P = radix(N, s), pstride(N, s)
        NB = N // R
        rlin = NB % 32 == 0 or 32 % NB == 0
        wlin = P % 32 == 0 or (32 % P == 0 and (32 % (P * R) == 0 or (P * R) % 32 == 0))
        for i in range(NB):
            k = i % P
            base = (i - k) * R + k
            for j in range(R):
                if rlin:
                    assert fpi(i + j * NB) == fpi(i) + pstep(j * NB)
                if wlin:
                    assert fpi(base + j * P) == fpi(base) + pstep(j * P)
        prod *= R
    assert prod == N
    # the layout is a bijection onto [0, N + N/32)
    assert sorted(set(fpi(n) for n in range(N))) == sorted(fpi(n) for n in range(N))
    assert max(fpi(n) for n in range(N)) < N + N // 32


def test_first_stages_are_conflict_free():
    # 32 lanes of one LDS pass (8-byte elements, 32 bank pairs): the first
    # radix-8 stage writes 8 i + j, contiguous accesses read base + t
    for j in range(8):
        assert len({fpi(8 * i + j) % 32 for i in range(32)}) == 32
    for base in (0, 32, 96, 640):
        assert len({fpi(base + t) % 32 for t in range(32)}) == 32


# Plans for TL threads per line: a power of two whose plan ends in {4, 4}
# ends in one radix-16 stage instead when N / 16 == TL.
def use16(n, tl):
    return not has3(n) and log2m(n) % 3 == 1 and log2m(n) >= 4 and n // 16 == tl


def plan(n, tl):
    r = [radix(n, s) for s in range(nstages(n))]
    if use16(n, tl):
        assert r[-2:] == [4, 4]
        r = r[:-2] + [16]
    return r


def test_padded_twiddles_spread_the_strided_reads():
    # the twiddle reads j k N / (P R) of a stage with P = 8 land on two bank
    # pairs in the plain layout, on distinct ones in the padded layout
    N = 1024
    for j in range(1, 8):
        idx = [j * (lane % 8) * (N // 64) for lane in range(32)]
        assert len({a % 32 for a in set(idx)}) <= 2
        assert len({fpi(a) % 32 for a in set(idx)}) == len(set(idx))


def stockham(x, radices, inverse=False):
    """The kernels' Stockham stages in NumPy: butterfly i reads
    x[i + j N/R], multiplies input j by W_{PR}^{j (i mod P)}, takes an
    R-point DFT and writes output j to (i - i mod P) R + i mod P + j P."""
    N = len(x)
    sgn = 1.0 if inverse else -1.0
    x = x.astype(np.complex128)
    P = 1
    for R in radices:
        NB = N // R
        y = np.empty_like(x)
        for i in range(NB):
            k = i % P
            v = np.array([x[i + j * NB] * np.exp(sgn * 2j * np.pi * j * k / (P * R))
                          for j in range(R)])
            out = np.array([np.sum(v * np.exp(sgn * 2j * np.pi * np.arange(R) * q / R))
                            for q in range(R)])
            base = (i - k) * R + k
            for j in range(R):
                y[base + j * P] = out[j]
        x = y
        P *= R
    return x


@pytest.mark.parametrize("N,TL", [(1024, 64), (1024, 128), (1024, 32), (512, 32), (128, 8),
                                  (192, 16), (2048, 256)])
def test_thread_plans(N, TL):
    r = plan(N, TL)
    assert int(np.prod(r)) == N
    assert (16 in r) == use16(N, TL)
    # the radix-16 stage's reads (stride N/16) and writes (P = N/16) are
    # contiguous across lanes and base-plus-step in the padded layout
    if use16(N, TL):
        R, P = 16, N // 16
        NB = N // R
        for i in range(NB):
            base = (i - i % P) * R + i % P
            for j in range(R):
                assert fpi(i + j * NB) == fpi(i) + pstep(j * NB)
                assert fpi(base + j * P) == fpi(base) + pstep(j * P)
    rng = np.random.default_rng(N + TL)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    np.testing.assert_allclose(stockham(x, r), np.fft.fft(x), rtol=0, atol=1e-9 * N)
    np.testing.assert_allclose(stockham(x, r, inverse=True), np.fft.ifft(x) * N, rtol=0,
                               atol=1e-9 * N)


def test_which_kernels_take_the_radix16_plan():
    # threads per line of the kernels: row passes pow2_floor(N / 8), column
    # passes 512 / (16, 8 or 4 columns), batched column passes 256 / (16 or 8)
    def pow2_floor(n):
        return 1 if n <= 1 else 2 * pow2_floor(n // 2)
    sizes = [64, 128, 192, 256, 384, 512, 1024, 2048]
    pairs = set()
    for n in sizes:
        pairs.add(("rows", n, pow2_floor(n // 8)))
        pairs.add(("cols", n, 512 // (4 if n >= 2048 else 8 if n >= 1024 else 16)))
        if n <= 1024:
            pairs.add(("cols2d", n, 256 // (8 if n >= 384 else 16)))
    assert {(k, n, tl) for k, n, tl in pairs if use16(n, tl)} == {("cols", 1024, 64)}
