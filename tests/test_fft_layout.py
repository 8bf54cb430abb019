"""Host-side check of the padded LDS line layout the frame FFTs use: element
n of a line sits at n + n/32, and the Stockham stages address it as a
per-butterfly base plus compile-time steps wherever the stride allows.  The
stage plan (radix 8, then 4 or 2, one radix-3 stage first for 3 * 2^a) and
the conditions below restate the kernels' compile-time rules; the test
checks that every base-plus-step address equals the element-wise one."""

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
