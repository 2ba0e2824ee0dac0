"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: bit-exact on integer data for the Hough transforms (every partial sum stays below 2^24);
relative RMSE <= 1e-5 for float32 reconstructions and filters against the FP64 oracle.
Inputs are seeded and synthetic (fbp_inputs); both sides see the same float32 values.
"""
import math

import numpy as np
import pytest
import torch

import fbp_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

RTOL_RMSE = 1e-5
# fixed coefficients (orders 1..8), stable, ramp-like; parity does not depend on their quality
COEF = {
    1: ([0.1344], [0.4832]),
    2: ([0.12372452, -0.12372452], [-0.17164439, -0.13239954]),
    3: ([0.12496065, -0.22928063, 0.10431998], [-1.02368667, 0.00172808, 0.09470333]),
    4: ([0.12493199, -0.122976, -0.0727046, 0.07074861],
        [-0.17279862, -0.72164016, 0.07148985, 0.04270461]),
}


def _coef(order, groups=1, seed=0, balanced=False):
    """FP64 coefficients, as the ABI takes them; both sides get the same values.  The fixed
    sets of orders 2-4 have sum(b) = 0 (zero response at zero frequency, as the ramp): the
    kernels' first-difference numerator then has no remainder term.  Random sets (orders 5-8,
    several groups) are unbalanced, with a remainder, unless `balanced`, which removes the mean
    of each group's b."""
    if order in COEF and groups == 1:
        b, a = COEF[order]
        return np.array(b), np.array(a)
    g = np.random.default_rng(seed + 31 * order + groups)
    bs, as_ = [], []
    for _ in range(groups):
        poles = g.uniform(-0.8, 0.8, size=order)
        as_.append(np.poly(poles)[1:])
        b = g.normal(size=order) * 0.05
        b[0] = 0.125
        if balanced:
            b = b - b.mean()
        bs.append(b)
    return np.array(bs), np.array(as_)


def _coef32(order, groups=1, seed=0, balanced=False):
    """The same coefficients rounded to float32 (unbalanced by the rounding: the kernels add
    the remainder term)."""
    b, a = _coef(order, groups, seed, balanced)
    return b.astype(np.float32).astype(np.float64), a.astype(np.float32).astype(np.float64)


def _rel_rmse(got, ref):
    got = got.detach().cpu().to(torch.float64)
    ref = ref.to(torch.float64)
    return float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref))


def _phantom_lino(N, B, seed, disc=0.34):
    d = disc if N >= 64 else 0.25
    ells = I.random_ellipses(N, 10, seed, disc=d, batch=B)
    return I.linogram(ells, N).to(torch.float32)


# ---- exact integer Hough transforms --------------------------------------------------------

@pytest.mark.parametrize("N,B", [(4, 1), (8, 2), (16, 3), (32, 2), (64, 2), (128, 3), (256, 2),
                                 (512, 2), (1024, 1), (2048, 1)])
def test_backproject_integer_bit_exact(gpu_lib, N, B):
    api = gpu_lib
    P = I.random_int_array((B, 4, N, N), 0, 1000, seed=N + B).to(torch.float32)
    with api.fbp_plan(N, B, *_coef(2)) as plan:
        got = api.fht_backproject(plan, P.cuda())
        torch.cuda.synchronize()
    ref = O.fht_backproject(P.to(torch.float64))
    assert torch.equal(got.cpu().to(torch.float64), ref)


@pytest.mark.parametrize("N,B", [(4, 1), (16, 2), (64, 3), (256, 1), (1024, 1), (2048, 1)])
def test_forward_integer_bit_exact(gpu_lib, N, B):
    api = gpu_lib
    f = I.random_int_array((B, N, N), 0, 1000, seed=7 * N + B).to(torch.float32)
    with api.fbp_plan(N, B, *_coef(2)) as plan:
        got = api.fht_forward(plan, f.cuda())
        torch.cuda.synchronize()
    ref = O.fht_forward(f.to(torch.float64))
    assert torch.equal(got.cpu().to(torch.float64), ref)


@pytest.mark.parametrize("N", [2048])
def test_adjoint_identity_on_gpu(gpu_lib, N):
    api = gpu_lib
    x = I.random_int_array((1, N, N), 0, 1000, seed=1).to(torch.float32).cuda()
    y = I.random_int_array((1, 4, N, N), 0, 1000, seed=2).to(torch.float32).cuda()
    with api.fbp_plan(N, 1, *_coef(2)) as plan:
        hx = api.fht_forward(plan, x)
        hty = api.fht_backproject(plan, y)
        torch.cuda.synchronize()
    lhs = (hx.double() * y.double()).sum().item()
    rhs = (x.double() * hty.double()).sum().item()
    assert lhs == rhs


# ---- recursive filter ------------------------------------------------------------------------

@pytest.mark.parametrize("N,order,groups", [(32, 2, 1), (64, 1, 1), (128, 2, 1), (256, 3, 1),
                                            (256, 4, 8), (512, 5, 1), (1024, 2, 1),
                                            (1024, 4, 8), (2048, 2, 1), (128, 8, 4),
                                            (64, 6, 2), (128, 7, 1), (16, 2, 1), (8, 3, 1)])
def test_filter_matches_oracle(gpu_lib, N, order, groups):
    api = gpu_lib
    B = 2
    P = torch.randn(B, 4, N, N, generator=torch.Generator().manual_seed(N + order),
                    dtype=torch.float64).to(torch.float32)
    b, a = _coef(order, groups)
    with api.fbp_plan(N, B, b, a) as plan:
        got = api.fbp_filter(plan, P.cuda())
        torch.cuda.synchronize()
    ref = O.filter_linogram(P.to(torch.float64), torch.tensor(b), torch.tensor(a))
    assert _rel_rmse(got, ref) < RTOL_RMSE


@pytest.mark.parametrize("flags", [1, 2, 4, 6])
def test_filter_flags(gpu_lib, flags):
    api = gpu_lib
    N, B = 128, 1
    P = torch.randn(B, 4, N, N, generator=torch.Generator().manual_seed(flags),
                    dtype=torch.float64).to(torch.float32)
    b, a = _coef(2)
    with api.fbp_plan(N, B, b, a, flags=flags) as plan:
        got = api.fbp_filter(plan, P.cuda())
        torch.cuda.synchronize()
    ref = O.filter_linogram(P.to(torch.float64), torch.tensor(b), torch.tensor(a),
                            scale=not (flags & 1), input_is_fht=bool(flags & 2),
                            windowed=not (flags & 4))
    assert _rel_rmse(got, ref) < RTOL_RMSE


def test_filter_in_place(gpu_lib):
    api = gpu_lib
    N, B = 256, 2
    P = _phantom_lino(N, B, 5)
    b, a = _coef(2)
    with api.fbp_plan(N, B, b, a) as plan:
        x = P.cuda()
        api.fbp_filter(plan, x, x)
        torch.cuda.synchronize()
    ref = O.filter_linogram(P.to(torch.float64), torch.tensor(b), torch.tensor(a))
    assert _rel_rmse(x, ref) < RTOL_RMSE


# ---- the method end to end ------------------------------------------------------------------

def _max_rel(got, ref):
    """Largest per-pixel error over the largest reference magnitude."""
    got = got.detach().cpu().to(torch.float64)
    return float((got - ref).abs().max() / ref.abs().max())


@pytest.mark.parametrize("N,B,order", [(8, 1, 2), (16, 2, 2), (32, 2, 2), (64, 2, 3),
                                       (128, 3, 2), (256, 2, 2), (512, 2, 4), (1024, 2, 2),
                                       (1024, 1, 3), (1024, 1, 4), (2048, 1, 2), (2048, 1, 3),
                                       (2048, 1, 4)])
def test_reconstruct_matches_oracle(gpu_lib, N, B, order):
    """FP64 coefficients on both sides (the balanced sets run in first-difference form)."""
    api = gpu_lib
    P = _phantom_lino(N, B, seed=N)
    b, a = _coef(order)
    with api.fbp_plan(N, B, b, a) as plan:
        got = api.fbp_reconstruct(plan, P.cuda())
        torch.cuda.synchronize()
    ref = O.fbp_fht(P.to(torch.float64), torch.tensor(b), torch.tensor(a))
    assert _rel_rmse(got, ref) < RTOL_RMSE
    assert _max_rel(got, ref) < 10 * RTOL_RMSE


def _fp32_bar(a):
    """The float32 bar of a recursive filter: the relative error a float32 recursion carries,
    its per-step rounding (2^-24) amplified by the l1 norm of the all-pole part's impulse
    response (the noise gain of 1/A(z)), twice over; never below RTOL_RMSE.  For poles close
    to 1 (the order-4 frequency-domain fit: 0.9946 and 0.9357, DC gain 1/A(1) about 4000)
    this is well above 1e-5: a sequential float32 recursion of that filter in the same
    first-difference form lands 2.3e-4 from the FP64 result at N = 512."""
    h = np.zeros(1 << 16)
    h[0] = 1.0
    for n in range(1, len(h)):
        h[n] = -sum(a[k] * h[n - 1 - k] for k in range(min(len(a), n)))
    return max(RTOL_RMSE, 2.0 * 2.0 ** -24 * float(np.abs(h).sum()))


def _scan_depth(a, L):
    """Scan levels a chunk of L samples needs: the first j where ||M^(L 2^j)|| / (1 - ||M^L||)
    is at most 2^-30, M the companion matrix of 1/A(z) over the last K outputs, infinity norm;
    7 (every level) when ||M^L|| >= 1."""
    K = len(a)
    M = np.zeros((K, K))
    M[0, :] = -np.asarray(a, dtype=np.float64)
    M[1:, :-1] = np.eye(K - 1)
    n = [np.abs(np.linalg.matrix_power(M, L << j)).sum(1).max() for j in range(7)]
    if not n[0] < 1.0:
        return 7
    return next((j for j in range(7) if n[j] / (1.0 - n[0]) <= 2.0 ** -30), 7)


@pytest.mark.parametrize("N,order,frequency", [(1024, 2, False), (1024, 4, False), (512, 4, False),
                                               (1024, 3, True), (1024, 4, True), (512, 4, True)])
def test_reconstruct_scan_depths_match_oracle(gpu_lib, N, order, frequency):
    """The plan runs as many levels of the chunk-state scan as its coefficients need (none for
    the order-2 time-domain fit, whose chunk transition has norm 3e-11; 3 of 5 for the order-4
    one; all for the frequency-domain fits, with poles within 1 - 2/L of the unit circle).
    The depth the plan reports is the one numpy finds for its chunks of 32 samples.  Each
    image against the FP64 oracle, which filters whole rows, to the filter's float32 bar."""
    api = gpu_lib
    P = _phantom_lino(N, 2, seed=N + 7 * order + frequency)
    b, a, _ = api.fbp_fit_ramp_iir(order, N if frequency else min(N, 512), dc_zero=True,
                                   frequency=frequency)
    want = {(2, False): 0, (4, False): 3}.get((order, frequency), 7)
    assert _scan_depth(a, 32) == want
    with api.fbp_plan(N, 2, b, a) as plan:
        assert plan.filter_info() == {"chunk": 32, "scan_levels": want, "first_levels": want,
                                      "remainder": False}
        got = api.fbp_reconstruct(plan, P.cuda())
        torch.cuda.synchronize()
    ref = O.fbp_fht(P.to(torch.float64), torch.tensor(b), torch.tensor(a))
    bar = _fp32_bar(a)
    assert _rel_rmse(got, ref) < bar
    assert _max_rel(got, ref) < 10 * bar


@pytest.mark.parametrize("N,order,balanced", [(512, 5, True), (512, 6, False), (512, 8, True),
                                              (1024, 5, False), (1024, 6, True),
                                              (1024, 8, False), (1024, 8, True)])
def test_reconstruct_high_orders_fused(gpu_lib, N, order, balanced):
    """Orders 5..8 through the fused first pass (the order-8 kernel, zero-padded for 5..7),
    in both numerator forms, against the FP64 oracle: relative RMSE and per-pixel maximum."""
    api = gpu_lib
    P = _phantom_lino(N, 2, seed=N + order)
    b, a = _coef(order, balanced=balanced)
    with api.fbp_plan(N, 2, b, a) as plan:
        got = api.fbp_reconstruct(plan, P.cuda())
        torch.cuda.synchronize()
    ref = O.fbp_fht(P.to(torch.float64), torch.tensor(b), torch.tensor(a))
    assert _rel_rmse(got, ref) < RTOL_RMSE
    assert _max_rel(got, ref) < 10 * RTOL_RMSE


def test_reconstruct_learned_filter_shape(gpu_lib):
    """The learned filter's launch shape: N = 1024, order 4, 8 angle groups with sum(b) = 0 (the
    order-4 first-pass kernel with one coefficient set per group, in first-difference form),
    two slices of 30 ellipses with Poisson noise at 1e4 photons."""
    api = gpu_lib
    N, B = 1024, 2
    ells = I.random_ellipses(N, 30, seed=55, batch=B)
    P = I.poisson_noisy(I.linogram(ells, N), 1e4, seed=56).to(torch.float32)
    b, a = _coef(4, groups=8, balanced=True)
    with api.fbp_plan(N, B, b, a) as plan:
        got = api.fbp_reconstruct(plan, P.cuda())
        torch.cuda.synchronize()
    ref = O.fbp_fht(P.to(torch.float64), torch.tensor(b), torch.tensor(a))
    assert _rel_rmse(got, ref) < RTOL_RMSE
    assert _max_rel(got, ref) < 10 * RTOL_RMSE


def test_reconstruct_4096_rows_over_two_waves(gpu_lib):
    """N = 4096: a row has 128 chunks of 32 samples, so pass 0 spreads each row over two waves
    and joins their chunk scans through LDS (the filter alone keeps 64-sample chunks).  Orders
    1..4 with FP64 coefficients against the FP64 oracle, fused and as the filter followed by
    the back projection; the two float32 chunkings also agree with each other."""
    api = gpu_lib
    N = 4096
    ells = I.random_ellipses(N, 10, 4096, disc=0.34, batch=1)
    P = I.linogram(ells, N, device="cuda", dtype=torch.float32)
    Pd = P.cpu().to(torch.float64)
    for order in (1, 2, 3, 4):
        b, a = _coef(order)
        with api.fbp_plan(N, 1, b, a) as plan:
            got = api.fbp_reconstruct(plan, P).clone()
            two_step = api.fht_backproject(plan, api.fbp_filter(plan, P))
            torch.cuda.synchronize()
        assert _rel_rmse(got, two_step.cpu().to(torch.float64)) < 1e-6, order
        ref = O.fbp_fht(Pd, torch.tensor(b), torch.tensor(a))
        assert _rel_rmse(got, ref) < RTOL_RMSE, order
        assert _rel_rmse(two_step, ref) < RTOL_RMSE, order


def test_forward_4096_sampled_rows_bit_exact(gpu_lib):
    """Forward transform at the largest size on integers <= 250 (every partial sum below 2^24):
    sampled rows of every class against the definition lino[q][t][s] = sum over y of the
    class-q frame's row y at column (s + D[t, y]) mod N (eq 16-17)."""
    api = gpu_lib
    N = 4096
    f = I.random_int_array((1, N, N), 0, 250, seed=4097).to(torch.float32)
    with api.fbp_plan(N, 1, *_coef(2)) as plan:
        got = api.fht_forward(plan, f.cuda())
        torch.cuda.synchronize()
    D = O.dyadic_shift(N)
    fd = f[0].to(torch.float64)
    y = torch.arange(N)
    for q in range(4):
        fr = O.to_frame(fd, q)
        for t in (0, 1, 2047, 4095):
            for s0 in (0, 1777, 4095 - 7):
                s = torch.arange(s0, s0 + 8)
                cols = (s[None, :] + D[t][:, None]) % N            # [y, 8]
                ref = torch.gather(fr, 1, cols).sum(0)
                assert torch.equal(got[0, q, t, s0:s0 + 8].cpu().to(torch.float64), ref), (q, t, s0)


@pytest.mark.parametrize("N,flags", [(512, 4), (1024, 4), (1024, 1), (1024, 2)])
def test_reconstruct_flags_on_the_fused_first_pass(gpu_lib, N, flags):
    """The fused first pass (filter, level 0 in registers, radix-4 stages, direct stores) with
    the plan flags: 4 keeps the rows at shift 0 (no window rotation), 1 skips c_t, 2 multiplies
    in one more k_t."""
    api = gpu_lib
    P = _phantom_lino(N, 1, seed=N + flags)
    b, a = _coef(2)
    with api.fbp_plan(N, 1, b, a, flags=flags) as plan:
        got = api.fbp_reconstruct(plan, P.cuda())
        torch.cuda.synchronize()
    ref = O.fbp_fht(P.to(torch.float64), torch.tensor(b), torch.tensor(a),
                    scale=not (flags & 1), input_is_fht=bool(flags & 2),
                    windowed=not (flags & 4))
    assert _rel_rmse(got, ref) < RTOL_RMSE


def test_coefficient_rounding_sensitivity(gpu_lib):
    """The reconstruction amplifies an offset in the filter's zero-frequency response by about
    N.  With FP64 balanced coefficients (sum(b) = 0) the first-difference numerator keeps that
    response exactly zero, and the bar holds at orders 2 and 4.  Fed float32-rounded
    coefficients (sum(b) a few ulps off zero: a remainder term s = sum(b), rounded once), it
    matches an oracle given the same rounded values."""
    api = gpu_lib
    N, B = 512, 1
    P = _phantom_lino(N, B, seed=N)
    for order in (2, 4):
        for coef in (_coef, _coef32):
            b, a = coef(order)
            with api.fbp_plan(N, B, b, a) as plan:
                got = api.fbp_reconstruct(plan, P.cuda())
                torch.cuda.synchronize()
            ref = O.fbp_fht(P.to(torch.float64), torch.tensor(b), torch.tensor(a))
            assert _rel_rmse(got, ref) < RTOL_RMSE, (order, coef.__name__)


def test_numerator_form_switch_makes_graphs_stale(gpu_lib):
    """Coefficients that change between balanced and unbalanced add or drop the remainder term
    of the numerator, which a captured graph has compiled in: its launch is refused until it
    is captured again.  An update that keeps the form is seen by the graph.  A nearly balanced
    numerator (sum(b) = 1e-3 b_0) still meets the bar: its remainder is rounded once."""
    api = gpu_lib
    N, B = 256, 1
    P = _phantom_lino(N, B, seed=3).cuda()
    b, a = _coef(4)
    with api.fbp_plan(N, B, b, a) as plan:
        img = torch.empty(B, N, N, device="cuda")
        g = api.fbp_graph_create([plan], [P], [img])
        b2 = b * 1.5                                       # still balanced
        api.fbp_plan_set_coefficients(plan, b2, a)
        g.launch()
        torch.cuda.synchronize()
        ref = O.fbp_fht(P.cpu().to(torch.float64), torch.tensor(b2), torch.tensor(a))
        assert _rel_rmse(img, ref) < RTOL_RMSE
        b3 = b2.copy()
        b3[0] += 1e-3 * b3[0]                              # unbalanced: remainder term
        api.fbp_plan_set_coefficients(plan, b3, a)
        with pytest.raises(api.FbpError) as e:
            g.launch()
        assert e.value.code == -1
        g.close()
        got = api.fbp_reconstruct(plan, P)
        torch.cuda.synchronize()
        ref = O.fbp_fht(P.cpu().to(torch.float64), torch.tensor(b3), torch.tensor(a))
        assert _rel_rmse(got, ref) < RTOL_RMSE


def test_reconstruct_equals_filter_then_backproject(gpu_lib):
    api = gpu_lib
    N, B = 512, 2
    P = _phantom_lino(N, B, 9).cuda()
    with api.fbp_plan(N, B, *_coef(3)) as plan:
        fused = api.fbp_reconstruct(plan, P)
        split = api.fht_backproject(plan, api.fbp_filter(plan, P))
        torch.cuda.synchronize()
    assert _rel_rmse(fused, split.cpu().double()) < 1e-6


def test_reconstruct_grouped_coefficients(gpu_lib):
    api = gpu_lib
    N, B = 256, 2
    P = _phantom_lino(N, B, 11)
    b, a = _coef(4, groups=8)
    with api.fbp_plan(N, B, b, a) as plan:
        got = api.fbp_reconstruct(plan, P.cuda())
        torch.cuda.synchronize()
    ref = O.fbp_fht(P.to(torch.float64), torch.tensor(b), torch.tensor(a))
    assert _rel_rmse(got, ref) < RTOL_RMSE


def test_full_size_batch_sampled_parity(gpu_lib):
    """512 slices of N = 1024 (the benchmark's launch configuration); two slices checked."""
    api = gpu_lib
    N, B = 1024, 512
    lino, _ = I.volume_linogram(N, B, count=30, seed=3, device="cuda")
    b, a = _coef(2)
    with api.fbp_plan(N, B, b, a) as plan:
        img = api.fbp_reconstruct(plan, lino)
        torch.cuda.synchronize()
    for s in (0, 301):
        ref = O.fbp_fht(lino[s].cpu().to(torch.float64), torch.tensor(b), torch.tensor(a))
        assert _rel_rmse(img[s], ref) < RTOL_RMSE


# ---- edge cases and errors ----------------------------------------------------------------

def test_empty_batch_and_errors(gpu_lib):
    api = gpu_lib
    N = 64
    with api.fbp_plan(N, 2, *_coef(2)) as plan:
        z = torch.empty(0, 4, N, N, device="cuda")
        out = api.fbp_reconstruct(plan, z)
        assert out.shape == (0, N, N)
        with pytest.raises(api.FbpError) as e:
            api.fbp_reconstruct(plan, torch.zeros(3, 4, N, N, device="cuda"))
        assert e.value.code == -5
        with pytest.raises(ValueError):
            api.fbp_reconstruct(plan, torch.zeros(1, 4, N, N, device="cuda", dtype=torch.float64))
        with pytest.raises(ValueError):
            api.fbp_reconstruct(plan, torch.zeros(1, 4, N, N))
    with pytest.raises(api.FbpError) as e:
        api.fbp_plan(N, 1, [0.1, 0.1], [0.0, 1.5])
    assert e.value.code == -2


def test_plan_pass_structure(gpu_lib):
    api = gpu_lib
    expect = {4: [2], 64: [6], 128: [7], 256: [3, 5], 512: [4, 5], 1024: [5, 5],
              2048: [2, 4, 5], 4096: [2, 5, 5]}
    for N, lv in expect.items():
        with api.fbp_plan(N, 1, *_coef(2)) as plan:
            assert plan.passes() == lv


def test_max_size_4096(gpu_lib):
    api = gpu_lib
    N = 4096
    P = I.random_int_array((1, 4, N, N), 0, 250, seed=4096).to(torch.float32)
    with api.fbp_plan(N, 1, *_coef(2)) as plan:
        got = api.fht_backproject(plan, P.cuda())
        torch.cuda.synchronize()
    # sampled rows against the definition: image row y = sum over classes and slopes
    D = O.dyadic_shift(N)
    Pd = P[0].to(torch.float64)
    x = torch.arange(N)
    for y in (0, 1234, 4095):
        ref = torch.zeros(N, dtype=torch.float64)
        # class 0 contributes sum_t P0[t][(x - D[t,y]) mod N]; class 1 mirrored in x
        idx = (x[None, :] - D[:, y][:, None]) % N
        ref += torch.gather(Pd[0], 1, idx).sum(0)
        ref += torch.gather(Pd[1], 1, idx).sum(0).flip(0)
        # classes 2, 3 contribute through the transpose: image[y][x] gets FHT^T(P2)[x][y]
        idxT = (y - D[:, x]) % N                      # [t, x]
        ref += torch.gather(Pd[2], 1, idxT).sum(0)
        idx3 = ((N - 1 - y) - D[:, x]) % N
        ref += torch.gather(Pd[3], 1, idx3).sum(0)
        assert torch.equal(got[0, y].cpu().to(torch.float64), ref)


# ---- direct FBP comparator ------------------------------------------------------------------

@pytest.mark.parametrize("N,P", [(64, 256), (128, 512)])
def test_direct_fbp_comparator_matches_oracle(gpu_lib, N, P):
    api = gpu_lib
    ells = I.random_ellipses(N, 10, seed=N)
    sino = I.parallel_sinogram(ells, N, P).to(torch.float32)
    got = api.fbp_direct_parallel(sino[None].cuda(), N)
    torch.cuda.synchronize()
    ref = O.fbp_direct_parallel(sino.to(torch.float64), N)
    assert _rel_rmse(got[0], ref) < 1e-4
