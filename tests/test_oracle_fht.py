"""Pins of the oracle's dyadic patterns, Fast Hough Transform and its transpose (CPU only).

Independent checks: hand-derived patterns, a bitwise closed form of the pattern offsets,
brute-force dense sums on integers (bit-exact), the adjoint identity, the mirror identity of
eq 19, the Radon invariant of Sec. 4.2 and the straight-line approximation bound.
"""
import math
import os

import pytest
import torch

import fbp_inputs as I
import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _bits_closed_form(N):
    n = N.bit_length() - 1
    D = torch.zeros(N, N, dtype=torch.int64)
    for t in range(N):
        for y in range(N):
            v = 0
            for a in range(n):
                for b in range(n):
                    ya = (y >> a) & 1
                    tb = (t >> b) & 1
                    if a + b >= n:
                        v += (1 << (a + b - n)) * ya * tb
                    elif a + b == n - 1:
                        v += ya * tb
            D[t, y] = v
    return D


def test_dyadic_patterns_match_hand_derivation():
    rows = {}
    for line in open(os.path.join(GOLD, "dyadic_patterns_n4_n8.txt")):
        if line.startswith("#") or not line.strip():
            continue
        head, vals = line.split(":")
        N, t = (int(v) for v in head.split())
        rows.setdefault(N, {})[t] = [int(v) for v in vals.split()]
    for N, tab in rows.items():
        ref = torch.tensor([tab[t] for t in range(N)])
        assert torch.equal(O.dyadic_shift(N), ref)


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 32, 64, 128])
def test_dyadic_closed_form_and_properties(N):
    D = O.dyadic_shift(N)
    assert torch.equal(D, _bits_closed_form(N))
    assert torch.equal(D, D.T)                       # symmetric
    assert (D[:, 0] == 0).all()
    assert torch.equal(D[:, -1], torch.arange(N))
    if N > 1:
        steps = D[:, 1:] - D[:, :-1]
        assert ((steps == 0) | (steps == 1)).all()   # a connected digital line
        t = torch.arange(N, dtype=torch.float64)
        dev = (D.double() - t[:, None] * t[None, :] / (N - 1)).abs().max()
        assert float(dev) <= math.log2(N) / 6 + 1e-12


def _brute_fht(img, D):
    N = img.shape[-1]
    H = torch.zeros_like(img)
    for t in range(N):
        for s in range(N):
            H[t, s] = sum(img[y, (s + D[t, y]) % N] for y in range(N))
    return H


def _brute_fht_T(P, D):
    N = P.shape[-1]
    R = torch.zeros_like(P)
    for y in range(N):
        for x in range(N):
            R[y, x] = sum(P[t, (x - D[t, y]) % N] for t in range(N))
    return R


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 32])
def test_fht_and_transpose_match_brute_force_exactly(N):
    D = O.dyadic_shift(N)
    img = I.random_int_array((N, N), 0, 1000, seed=100 + N)
    P = I.random_int_array((N, N), 0, 1000, seed=200 + N)
    assert torch.equal(O.fht(img), _brute_fht(img, D))
    assert torch.equal(O.fht_T(P), _brute_fht_T(P, D))


@pytest.mark.parametrize("N", [64, 256])
def test_fht_adjoint_identity_exact(N):
    x = I.random_int_array((2, N, N), 0, 1000, seed=1)
    y = I.random_int_array((2, N, N), 0, 1000, seed=2)
    lhs = (O.fht(x) * y).sum()
    rhs = (x * O.fht_T(y)).sum()
    assert float(lhs) == float(rhs)


@pytest.mark.parametrize("N", [8, 64, 256])
def test_transpose_is_mirrored_forward_exact(N):
    # discrete eq 19: back projection = forward projection with one coordinate reversed
    P = I.random_int_array((N, N), 0, 1000, seed=3)
    mirror = lambda a: torch.roll(a.flip(-1), 1, dims=-1)   # a[(-x) mod N]  # noqa: E731
    assert torch.equal(O.fht_T(P), mirror(O.fht(mirror(P))))


@pytest.mark.parametrize("N", [16, 128])
def test_radon_invariant(N):
    img = I.random_int_array((N, N), 0, 1000, seed=4)
    H = O.fht(img)
    assert torch.equal(H.sum(-1), torch.full((N,), float(img.sum()), dtype=torch.float64))


def test_pattern_image_projects_to_a_single_bin():
    N = 32
    D = O.dyadic_shift(N)
    for t, s in [(0, 5), (7, 30), (31, 0), (19, 13)]:
        img = torch.zeros(N, N, dtype=torch.float64)
        for y in range(N):
            img[y, (s + D[t, y]) % N] = 1.0
        H = O.fht(img)
        assert H[t, s] == N
        assert H.sum() == N * N


def test_frames_are_permutation_inverses_and_follow_class_lines():
    N = 16
    f = I.random_int_array((N, N), 0, 1000, seed=5)
    for q in range(4):
        assert torch.equal(O.from_frame(O.to_frame(f, q), q), f)
    D = O.dyadic_shift(N)
    H = O.fht_forward(f)
    # class lines in image indices (x = column, y = row), see the fbp_inputs docstring
    for t, s in [(0, 0), (5, 9), (15, 3), (10, 15)]:
        v0 = sum(f[y, (s + D[t, y]) % N] for y in range(N))
        v1 = sum(f[y, N - 1 - (s + D[t, y]) % N] for y in range(N))
        v2 = sum(f[(s + D[t, x]) % N, x] for x in range(N))
        v3 = sum(f[N - 1 - (s + D[t, x]) % N, x] for x in range(N))
        assert [float(H[q, t, s]) for q in range(4)] == [float(v0), float(v1), float(v2), float(v3)]


@pytest.mark.parametrize("N", [16, 128])
def test_backproject_is_adjoint_of_forward(N):
    f = I.random_int_array((N, N), 0, 1000, seed=6)
    P = I.random_int_array((4, N, N), 0, 1000, seed=7)
    assert float((O.fht_forward(f) * P).sum()) == float((f * O.fht_backproject(P)).sum())


def test_add_count_model():
    assert O.fht_add_count(1024) == 1024 * 1024 * 10
    with pytest.raises(ValueError):
        O.fht(torch.zeros(6, 6))
