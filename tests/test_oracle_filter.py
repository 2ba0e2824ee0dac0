"""Pins of the oracle's ramp filter, recursive filters and row geometry (CPU only).

Each check is independent of the oracle's own code: numerical quadrature of eq 6, the printed
sinc form of eq 6, scipy's lfilter and residuez, exact sums, and symmetry identities.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.signal
import torch

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_ramp_taps_equal_eq6_sinc_form():
    rows = [l.split() for l in open(os.path.join(GOLD, "ramp_eq6.txt")) if not l.startswith("#")]
    n = torch.tensor([int(r[0]) for r in rows])
    ref = torch.tensor([float(r[1]) for r in rows], dtype=torch.float64)
    assert torch.allclose(O.ramp_taps(n), ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 7, 10, 13])
def test_ramp_taps_equal_band_limited_integral(n):
    # eq 6: h(n) = 2 * int_0^{1/2} |w| cos(2 pi w n) dw (imaginary parts cancel)
    val, err = scipy.integrate.quad(lambda w: 2 * w * math.cos(2 * math.pi * w * n), 0, 0.5,
                                    epsabs=1e-14, epsrel=1e-13, limit=200)
    assert abs(float(O.ramp_taps(n)) - val) < 1e-12


def test_ramp_dc_and_nyquist_response():
    n = torch.arange(-200001, 200002)
    h = O.ramp_taps(n)
    # |w| vanishes at w = 0 and equals 1/2 at the Nyquist frequency; the truncated tail of the
    # zero-frequency sum is about 1/(pi^2 L)
    assert abs(float(h.sum())) < 2.0 / (math.pi ** 2 * 200001)
    alt = torch.where(n % 2 == 0, 1.0, -1.0).to(torch.float64)
    assert abs(float((h * alt).sum()) - 0.5) < 2.0 / (math.pi ** 2 * 200001)


def test_causal_anticausal_split_rebuilds_ramp():
    L = 64
    hp = O.ramp_causal(L)
    full = O.ramp_taps(torch.arange(-(L - 1), L))
    rebuilt = torch.zeros(2 * L - 1, dtype=torch.float64)
    rebuilt[L - 1:] += hp            # h+ on n >= 0
    rebuilt[:L] += hp.flip(0)        # h- on n <= 0 (mirror of h+)
    assert torch.allclose(rebuilt, full, atol=1e-16)
    assert hp[0] == 0.125


@pytest.mark.parametrize("order", [1, 2, 3, 4, 6, 8])
def test_iir_causal_matches_lfilter(order):
    g = np.random.default_rng(order)
    b = g.normal(size=order) * 0.3
    poles = g.uniform(-0.9, 0.9, size=order)
    a = np.poly(poles)               # 1, a_1..a_Q with |poles| < 1
    x = g.normal(size=(3, 200))
    ref = scipy.signal.lfilter(b, a, x, axis=-1)
    got = O.iir_causal(torch.tensor(x), torch.tensor(b), torch.tensor(a[1:])).numpy()
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    ref_anti = scipy.signal.lfilter(b, a, x[:, ::-1], axis=-1)[:, ::-1]
    got_anti = O.iir_anticausal(torch.tensor(x), torch.tensor(b), torch.tensor(a[1:])).numpy()
    assert np.allclose(got_anti, ref_anti, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_iir_impulse_response_partial_fractions(order):
    g = np.random.default_rng(10 + order)
    b = g.normal(size=order)
    a = np.poly(g.uniform(-0.85, 0.85, size=order))
    r, p, k = scipy.signal.residuez(b, a)
    n = np.arange(60)
    closed = np.real(np.sum(r[:, None] * p[:, None] ** n[None, :], axis=0))
    for i, kk in enumerate(np.atleast_1d(k)):
        closed[i] += np.real(kk)
    got = O.iir_impulse_response(torch.tensor(b), torch.tensor(a[1:]), 60).numpy()
    assert np.allclose(got, closed, rtol=1e-10, atol=1e-12)


def test_iir_pair_response_is_symmetric():
    b = torch.tensor([0.125, -0.11, 0.02], dtype=torch.float64)
    a = torch.tensor([-0.3, -0.1, 0.05], dtype=torch.float64)
    x = torch.zeros(201, dtype=torch.float64)
    x[100] = 1.0
    y = O.iir_pair(x, b, a)
    assert torch.allclose(y, y.flip(0), atol=1e-15)
    # the pair's response equals g(|n|) with g(0) counted twice (eq 10-12)
    g = O.iir_impulse_response(b, a, 101)
    assert torch.allclose(y[100:], g + torch.cat([g[:1], torch.zeros(100, dtype=torch.float64)]))


def test_filter_with_identity_recursion_is_pure_row_scale():
    N = 32
    P = torch.randn(2, 4, N, N, dtype=torch.float64, generator=torch.Generator().manual_seed(3))
    b = torch.tensor([0.5], dtype=torch.float64)
    a = torch.tensor([0.0], dtype=torch.float64)
    out = O.filter_linogram(P, b, a)
    # each pass returns 0.5 x, the pair returns x; then the row scale
    ref = P * O.row_scale(N)[:, None]
    assert torch.allclose(out, ref, atol=1e-15)


def test_filter_with_full_fir_equals_numpy_convolution():
    # b = h+ over the whole row and no feedback turns the pair into the exact ramp FIR (eq 8)
    N = 32
    g = torch.Generator().manual_seed(4)
    P = torch.randn(4, N, N, dtype=torch.float64, generator=g)
    out = O.filter_linogram(P, O.ramp_causal(N), torch.zeros(1, dtype=torch.float64), scale=False)
    h = O.ramp_taps(torch.arange(-(N - 1), N)).numpy()
    sig = O.window_start(N).numpy()
    for q in range(4):
        for t in range(N):
            idx = (sig[t] + np.arange(N)) % N
            row = P[q, t].numpy()[idx]
            ref = np.convolve(row, h)[N - 1:2 * N - 1]
            assert np.allclose(out[q, t].numpy()[idx], ref, atol=1e-13)


def test_filter_is_self_adjoint():
    N = 16
    g = torch.Generator().manual_seed(5)
    x = torch.randn(4, N, N, dtype=torch.float64, generator=g)
    y = torch.randn(4, N, N, dtype=torch.float64, generator=g)
    b = torch.tensor([0.125, -0.1], dtype=torch.float64)
    a = torch.tensor([-0.2, -0.1], dtype=torch.float64)
    lhs = (O.filter_linogram(x, b, a) * y).sum()
    rhs = (x * O.filter_linogram_adjoint(y, b, a)).sum()
    assert abs(float(lhs - rhs)) < 1e-12 * float(lhs.abs() + 1)


def test_grouped_coefficients_select_rows():
    N = 16
    g = torch.Generator().manual_seed(6)
    P = torch.randn(4, N, N, dtype=torch.float64, generator=g)
    bs = torch.randn(8, 2, dtype=torch.float64, generator=g) * 0.1
    as_ = torch.randn(8, 2, dtype=torch.float64, generator=g) * 0.2
    out = O.filter_linogram(P, bs, as_)
    grp = O.row_groups(N, 8)
    assert grp[0, 0] == 0 and grp[3, N - 1] == 7 and grp[1, 0] == 2
    for gi in range(8):
        single = O.filter_linogram(P, bs[gi], as_[gi])
        sel = grp == gi
        assert torch.allclose(out[sel], single[sel])


def test_angle_weights_tile_half_circle():
    for N in [2, 8, 64, 1024]:
        w = O.angle_weights(N)
        assert abs(4 * float(w.sum()) - math.pi) < 1e-12
        assert (w > 0).all()
        th = O.angles(N)
        assert float(th[0]) == 0.0 and abs(float(th[-1]) - math.pi / 4) < 1e-15
        assert torch.allclose(O.stretch(N), 1 / torch.cos(th))


@pytest.mark.parametrize("N,disc", [(32, 0.25), (64, 0.3), (256, 0.34), (1024, 0.34)])
def test_window_covers_support_disc(N, disc):
    # every line through the disc of radius disc * N meets it at intercepts that lie inside
    # the row's window (reading R1), with one pixel to spare for the dyadic rounding
    sig = O.window_start(N)
    k = O.stretch(N)
    sc = (N - 1 - torch.arange(N)) / 2.0          # intercept of the line through the centre
    lo = sc - disc * N * k - 1
    hi = sc + disc * N * k + 1
    start = (N - 1 - torch.arange(N)) // 2 - N // 2
    assert torch.equal(start % N, sig)
    assert (lo >= start).all() and (hi <= start + N - 1).all()


@pytest.mark.parametrize("order", [2, 3, 4, 8])
def test_balanced_numerator_difference_form(order):
    """A numerator with sum(b) = 0 factors as B(z) = (1 - z^-1) C(z) with c_k = b_0 + .. + b_k
    (k < K - 1), the form the kernels take for such filters: filtering the first difference
    d[i] = x[i] - x[i-1] (zero before the window) by C and A gives the causal recursion of
    eq 9, and d'[i] = x[i] - x[i+1] gives the anticausal one (eq 13).  Zero response at zero
    frequency: a constant row gives an output that vanishes once the start transient decays."""
    g = np.random.default_rng(order)
    a = torch.tensor(np.poly(g.uniform(-0.7, 0.7, size=order))[1:])
    b = torch.tensor(g.normal(size=order))
    b = b - b.mean()
    c = torch.cumsum(b, 0)[:-1]
    x = torch.tensor(g.normal(size=(3, 200)))
    d = x - torch.nn.functional.pad(x, (1, 0))[:, :-1]
    yc = O.iir_causal(x, b, a)
    assert torch.allclose(O.iir_causal(d, c, a), yc, rtol=0, atol=1e-12 * float(yc.abs().max()))
    da = x - torch.nn.functional.pad(x, (0, 1))[:, 1:]
    ya = O.iir_anticausal(x, b, a)
    assert torch.allclose(O.iir_anticausal(da, c, a), ya, rtol=0,
                          atol=1e-12 * float(ya.abs().max()))
    flat = O.iir_pair(torch.ones(1, 400, dtype=torch.float64), b, a)[0]
    assert float(flat[150:250].abs().max()) < 1e-9
