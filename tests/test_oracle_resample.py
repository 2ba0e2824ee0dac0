"""Pins of the oracle's sinogram-to-linogram resampling (Sec. 4.2, eq 14; reading R16).

The geometry is held to the independent line parameterisation of the input generator and to
exact sinogram nodes; the interpolation to bilinear functions (reproduced exactly); the whole
map to exact linogram line integrals of analytic phantoms, with an error that falls as the
angular sampling grows.
"""
import math

import pytest
import torch

import fbp_inputs as I
import oracle as O


@pytest.mark.parametrize("N", [8, 32, 64])
def test_lines_match_the_generator_geometry(N):
    nx, ny, rho = O.linogram_lines(N)
    gx, gy, gr = I.linogram_line_params(N)
    assert torch.allclose(nx, gx, atol=1e-14) and torch.allclose(ny, gy, atol=1e-14)
    # the generator measures offsets from the corner: r = rho + (N/2)(nx + ny)
    assert torch.allclose(rho + 0.5 * N * (nx + ny), gr, atol=1e-12)


def test_axis_aligned_rows_are_exact_sinogram_rows():
    """t = 0 lines are sinogram rows at angle 0 (classes 0, 1) and pi/2 (classes 2, 3): with
    D = N their samples land on detector nodes, so the resampled values are copies."""
    N, P = 16, 8
    sino = torch.randn(P, N, generator=torch.Generator().manual_seed(1), dtype=torch.float64)
    lino = O.resample_sinogram(sino, N)
    s = torch.arange(N)
    assert torch.allclose(lino[0, 0], sino[0, s], atol=1e-12)            # x = s
    assert torch.allclose(lino[1, 0], sino[0, N - 1 - s], atol=1e-12)    # x = N-1-s
    assert torch.allclose(lino[2, 0], sino[P // 2, s], atol=1e-12)       # y = s
    assert torch.allclose(lino[3, 0], sino[P // 2, N - 1 - s], atol=1e-12)


def test_diagonal_rows_hit_the_45_degree_angles():
    """t = N - 1 (slope 1): class 0 lines have normal angle 3 pi/4, class 1 pi/4.  With a wide
    detector both folds of a cell (s and s - N) fall on it, so a cell holds 1 or 2."""
    N, P = 16, 16
    D = 3 * N
    sino = torch.zeros(P, D, dtype=torch.float64)
    sino[P // 4] = 1.0              # pi/4
    lino = O.resample_sinogram(sino, N)
    inside = lino[1, N - 1]
    assert torch.all((inside == 1.0) | (inside == 2.0)) and (inside == 2.0).any()
    assert lino[0, N - 1].abs().max() == 0.0   # 3 pi / 4 row is empty
    sino.zero_()
    sino[3 * P // 4] = 1.0
    lino = O.resample_sinogram(sino, N)
    assert lino[0, N - 1].abs().sum() > 0 and lino[1, N - 1].abs().max() == 0.0


def test_bilinear_functions_are_reproduced():
    N, P, D = 32, 40, 96
    i = torch.arange(P, dtype=torch.float64)[:, None]
    j = torch.arange(D, dtype=torch.float64)[None, :]
    f = lambda a, u: 0.3 + 0.02 * a - 0.01 * u + 0.001 * a * u    # noqa: E731
    sino = f(i, j)
    lino = O.resample_sinogram(sino, N)
    nx, ny, rho = O.linogram_lines(N)
    phi = torch.atan2(ny, nx)
    flip = phi < 0
    a = torch.where(flip, phi + math.pi, phi) * P / math.pi
    u = torch.where(flip, -rho, rho) + D / 2 - 0.5
    # stay inside the node grid (no angle wrap, no detector edge) where bilinear is exact
    ok = (a <= P - 1) & (u >= 0) & (u <= D - 1)
    expect = (f(a, u) * ok).sum(0)
    got_masked = O.resample_sinogram(sino, N)
    both = ok.all(0)
    assert both.sum() > 0.5 * both.numel()
    assert torch.allclose(got_masked[both], expect[both], atol=1e-12)
    assert torch.equal(lino, got_masked)


def test_angle_wrap_mirrors_the_detector():
    """Between angle P-1 and pi the lookup continues at angle 0 with the detector mirrored:
    a sinogram with sino(0, j) = g(j) and sino(i, j) = g(D-1-j) near pi is continuous."""
    N, P, D = 16, 64, 48
    g = torch.linspace(-1, 2, D, dtype=torch.float64) ** 2
    sino = g.flip(0).expand(P, D).clone()
    sino[0] = g                     # the same physical lines as angle pi
    lino = O.resample_sinogram(sino, N)
    ref = O.resample_sinogram(g.flip(0).expand(P, D).clone(), N)
    # class 0 with small slopes looks up angles in (P - 1, P): both give the same values
    assert torch.allclose(lino[0, 1:N // 8], ref[0, 1:N // 8], atol=1e-12)


def _gaussian_line_integrals(nx, ny, r, centre, sigma):
    """Exact integral of exp(-|x - centre|^2 / (2 sigma^2)) along x . n = r (corner origin)."""
    d = r - (centre[0] * nx + centre[1] * ny)
    return math.sqrt(2 * math.pi) * sigma * torch.exp(-d * d / (2 * sigma * sigma))


def _gaussian_errors(N, sigma, angle_counts, D):
    centre = torch.tensor([N / 2 + 9.3, N / 2 - 6.1], dtype=torch.float64)
    gx, gy, gr = I.linogram_line_params(N)          # the generator's own line geometry
    exact = _gaussian_line_integrals(gx, gy, gr, centre, sigma).sum(0)
    errs = []
    for P in angle_counts:
        th = torch.arange(P, dtype=torch.float64) * math.pi / P
        rj = torch.arange(D, dtype=torch.float64) - D / 2 + 0.5
        nx, ny = torch.cos(th)[:, None], torch.sin(th)[:, None]
        sino = _gaussian_line_integrals(nx, ny, rj[None, :] + 0.5 * N * (nx + ny), centre, sigma)
        lino = O.resample_sinogram(sino, N)
        errs.append(float(torch.linalg.vector_norm(lino - exact) /
                          torch.linalg.vector_norm(exact)))
    return errs


def test_resampled_smooth_object_converges_to_exact_linogram():
    """A Gaussian blob: exact line integrals on both geometries.  The error falls with the
    angle count down to the floor of linear interpolation along the unit-spaced detector,
    which scales as 1 / sigma^2."""
    N = 64
    e4 = _gaussian_errors(N, 4.0, (N // 2, 8 * N), 2 * N)
    assert e4[1] < 0.7 * e4[0] and e4[1] < 1e-2, e4
    e8 = _gaussian_errors(N, 8.0, (8 * N,), 2 * N)
    assert e8[0] < e4[1] / 3, (e4, e8)


def test_resampled_rows_keep_the_radon_invariant():
    """Every linogram row sums (times its sample spacing 1/k_t) to the object's mass (Sec. 4.2)."""
    N = 64
    ells = I.random_ellipses(N, 6, seed=5, disc=0.34)
    sino = I.parallel_sinogram(ells, N, 8 * N, n_det=4 * N)
    lino = O.resample_sinogram(sino, N)
    mass = float(I.phantom_image(ells, N, supersample=4).sum())
    rows = lino.sum(-1) / O.stretch(N)[None, :]
    assert torch.allclose(rows, torch.full_like(rows, mass), rtol=2e-2)
