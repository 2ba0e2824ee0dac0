"""End-to-end pins of the oracle and of the input generators against analytic phantoms (CPU)."""
import math

import pytest
import torch

import fbp_inputs as I
import oracle as O


def test_ellipse_line_integrals_match_numeric_quadrature():
    N = 64
    ells = I.random_ellipses(N, 6, seed=11)
    P = I.linogram(ells, N)
    g = torch.Generator().manual_seed(0)
    p = ells.params
    for _ in range(12):
        q = int(torch.randint(0, 4, (1,), generator=g))
        t = int(torch.randint(0, N, (1,), generator=g))
        s = int(torch.randint(0, N, (1,), generator=g))
        m = t / (N - 1)
        # walk the class line with arc-length step ds over a long parameter range
        u = torch.linspace(-2 * N, 2 * N, 400001, dtype=torch.float64)
        ds = float(u[1] - u[0]) * math.sqrt(1 + m * m)
        total = 0.0
        for shift in (0, -N):
            ss = s + shift
            if q == 0:
                X, Y = ss + 0.5 + m * (u - 0.5), u
            elif q == 1:
                X, Y = N - ss - 0.5 - m * (u - 0.5), u
            elif q == 2:
                X, Y = u, ss + 0.5 + m * (u - 0.5)
            else:
                X, Y = u, N - ss - 0.5 - m * (u - 0.5)
            val = torch.zeros_like(u)
            for e in range(p.shape[0]):
                cx, cy, a, b, phi, rho = p[e].tolist()
                dx, dy = X - cx, Y - cy
                uu = dx * math.cos(phi) + dy * math.sin(phi)
                vv = -dx * math.sin(phi) + dy * math.cos(phi)
                val += rho * (((uu / a) ** 2 + (vv / b) ** 2) <= 1).double()
            total += float(val.sum()) * ds
        assert abs(total - float(P[q, t, s])) < 2e-3 * max(1.0, abs(total))


def test_linogram_rows_preserve_mass_after_stretch():
    # Sec. 4.2: every linogram row sums to k_t times the image mass (the Radon invariant of
    # the line-integral normalisation)
    N = 128
    ells = I.random_ellipses(N, 10, seed=0)
    P = I.linogram(ells, N)
    mass = float(sum(math.pi * a * b * rho for _, _, a, b, _, rho in ells.params.tolist()))
    rows = P.sum(-1) / O.stretch(N)
    assert float((rows - mass).abs().max()) < 5e-3 * abs(mass)  # Riemann sum of a sampled projection


def test_direct_fbp_reconstructs_phantom():
    N = 128
    ells = I.random_ellipses(N, 10, seed=0)
    P = I.linogram(ells, N)
    ph = I.phantom_image(ells, N, supersample=4)
    mask = I.support_mask(N)
    rec = O.fbp_direct_linogram(P)
    assert O.relative_rmse(rec, ph, mask) < 0.04


def test_direct_fbp_of_uniform_disc_has_right_level():
    # a disc of density 1: the reconstruction is 1 inside, away from the rim (pins the weights)
    N = 128
    ells = I.EllipseSet(torch.tensor([[64.0, 64.0, 30.0, 30.0, 0.0, 1.0]], dtype=torch.float64))
    rec = O.fbp_direct_linogram(I.linogram(ells, N))
    c = torch.arange(N, dtype=torch.float64) + 0.5 - 64
    inner = (c[:, None] ** 2 + c[None, :] ** 2) < 20 ** 2
    assert abs(float(rec[inner].mean()) - 1.0) < 0.01
    sino = I.parallel_sinogram(ells, N, 4 * N)
    rec2 = O.fbp_direct_parallel(sino, N)
    assert abs(float(rec2[inner].mean()) - 1.0) < 0.01


def test_parallel_fbp_reconstructs_phantom():
    N = 128
    ells = I.random_ellipses(N, 10, seed=0)
    sino = I.parallel_sinogram(ells, N, 4 * N)
    ph = I.phantom_image(ells, N, supersample=4)
    rec = O.fbp_direct_parallel(sino, N)
    assert O.relative_rmse(rec, ph, I.support_mask(N)) < 0.06


def test_fht_fbp_with_exact_fir_approaches_direct_fbp_as_n_grows():
    # with b = h+ over the whole row and no feedback the recursive pair is the exact ramp, so
    # the only difference from the direct FBP is the dyadic rounding of the lines; it shrinks
    # relative to the image as N grows (the trend of the paper's RMSE-vs-size experiment)
    errs = []
    for N in [32, 64, 128]:
        ells = I.random_ellipses(N, 10, seed=0, disc=0.3)
        P = I.linogram(ells, N)
        mask = I.support_mask(N, disc=0.3)
        rec = O.fbp_fht(P, O.ramp_causal(N), torch.zeros(1, dtype=torch.float64))
        errs.append(O.relative_rmse(rec, O.fbp_direct_linogram(P), mask))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.08


def test_fht_fbp_of_fht_image_roundtrip_level():
    # back projection of the filtered forward transform of a smooth image returns it at the
    # right level when the input is in the linogram (row-sum) normalisation
    N = 64
    ells = I.EllipseSet(torch.tensor([[32.0, 32.0, 12.0, 9.0, 0.4, 1.0]], dtype=torch.float64))
    f = I.phantom_image(ells, N, supersample=4)
    H = O.fht_forward(f)
    rec = O.fbp_fht(H, O.ramp_causal(N), torch.zeros(1, dtype=torch.float64), input_is_fht=True)
    c = torch.arange(N, dtype=torch.float64) + 0.5 - 32
    inner = (c[:, None] ** 2 + c[None, :] ** 2) < 6 ** 2
    assert abs(float(rec[inner].mean()) - 1.0) < 0.05


def test_oracle_gradients_match_finite_differences():
    N = 16
    ells = I.random_ellipses(N, 4, seed=3, disc=0.3)
    P = I.linogram(ells, N).requires_grad_(True)
    b = torch.tensor([0.125, -0.1], dtype=torch.float64, requires_grad=True)
    a = torch.tensor([-0.2, -0.1], dtype=torch.float64, requires_grad=True)
    target = I.phantom_image(ells, N)
    loss = ((O.fbp_fht(P, b, a) - target) ** 2).sum()
    gP, gb, ga = torch.autograd.grad(loss, (P, b, a))
    # the gradient in the input is the adjoint chain: forward FHT, then the (self-adjoint) filter
    r = 2 * (O.fbp_fht(P.detach(), b, a) - target)
    gP_ref = O.filter_linogram_adjoint(O.fht_forward(r.detach()), b.detach(), a.detach())
    assert torch.allclose(gP, gP_ref, rtol=1e-10, atol=1e-10)
    eps = 1e-6
    for (param, grad) in ((b, gb), (a, ga)):
        for i in range(2):
            d = torch.zeros_like(param)
            d[i] = eps
            with torch.no_grad():
                if param is b:
                    lp = ((O.fbp_fht(P, b + d, a) - target) ** 2).sum()
                    lm = ((O.fbp_fht(P, b - d, a) - target) ** 2).sum()
                else:
                    lp = ((O.fbp_fht(P, b, a + d) - target) ** 2).sum()
                    lm = ((O.fbp_fht(P, b, a - d) - target) ** 2).sum()
            fd = float(lp - lm) / (2 * eps)
            assert abs(fd - float(grad[i])) < 1e-5 * max(1.0, abs(fd))


@pytest.mark.parametrize("depth", [8])
def test_ellipsoid_slices_shrink_towards_caps(depth):
    e3 = I.random_ellipsoids(64, depth, 5, seed=2)
    sl = I.ellipsoid_slices(e3, depth).params
    assert sl.shape == (depth, 5, 6)
    cz, sz = e3[:, 2], e3[:, 5]
    z = torch.arange(depth, dtype=torch.float64)[:, None] + 0.5
    inside = (z - cz).abs() < sz
    assert torch.equal(sl[..., 5] != 0, inside & (e3[:, 7] != 0))
    assert (sl[..., 2][inside] <= e3[:, 3].expand(depth, 5)[inside] + 1e-12).all()
