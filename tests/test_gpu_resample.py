"""Scanner input on the GPU: sinogram-to-linogram resampling (Sec. 4.2, eq 14) against the
FP64 oracle, and the reconstruction from a sinogram end to end.

Bars: float32 resampling within 1e-5 relative RMSE of the oracle (positions are float32 on
the GPU, so interpolation fractions differ by ~1e-7 of the detector range); rows that fall on
sinogram nodes are copied bit for bit; the composition equals the two calls one after the
other bit for bit and the FP64 oracle composition within 1e-5.
"""
import numpy as np
import pytest
import torch

import fbp_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

B2 = ([0.12372452, -0.12372452], [-0.17164439, -0.13239954])


def _coef():
    b, a = B2
    return (np.array(b, np.float32).astype(np.float64),
            np.array(a, np.float32).astype(np.float64))


def _rel(got, ref):
    got = got.detach().cpu().double()
    return float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref))


def _sino(N, P, D, B, seed):
    ells = I.random_ellipses(N, 10, seed, disc=0.34, batch=B)
    return I.parallel_sinogram(ells, N, P, n_det=D, device="cuda", dtype=torch.float32)


@pytest.mark.parametrize("N,P,D,B", [(16, 16, 16, 2), (64, 96, 101, 2), (256, 256, 384, 2),
                                     (1024, 1024, 1536, 1)])
def test_resample_matches_oracle(gpu_lib, N, P, D, B):
    api = gpu_lib
    sino = _sino(N, P, D, B, seed=N + P)
    got = api.fbp_resample_sinogram(sino, N)
    torch.cuda.synchronize()
    ref = O.resample_sinogram(sino.cpu().double(), N)
    assert _rel(got, ref) < 1e-5


def test_node_rows_are_copied_exactly(gpu_lib):
    api = gpu_lib
    N, P = 64, 32
    sino = torch.randn(1, P, N, generator=torch.Generator().manual_seed(3)).cuda()
    lino = api.fbp_resample_sinogram(sino, N)
    torch.cuda.synchronize()
    s = torch.arange(N, device="cuda")
    assert torch.equal(lino[0, 0, 0], sino[0, 0, s])
    assert torch.equal(lino[0, 1, 0], sino[0, 0, N - 1 - s])
    assert torch.equal(lino[0, 2, 0], sino[0, P // 2, s])
    assert torch.equal(lino[0, 3, 0], sino[0, P // 2, N - 1 - s])


@pytest.mark.parametrize("N,P,D", [(256, 512, 384), (1024, 1024, 1536)])
def test_reconstruct_from_sinogram(gpu_lib, N, P, D):
    api = gpu_lib
    sino = _sino(N, P, D, 2, seed=7)
    with api.fbp_plan(N, 2, *_coef()) as plan:
        img = api.fbp_reconstruct_sinogram(plan, sino)
        lino = api.fbp_resample_sinogram(sino, N)
        two_step = api.fbp_reconstruct(plan, lino)
        torch.cuda.synchronize()
        assert torch.equal(img, two_step)
    if N <= 256:
        b, a = _coef()
        ref = O.fbp_fht(O.resample_sinogram(sino.cpu().double(), N), torch.tensor(b),
                        torch.tensor(a))
        assert _rel(img, ref) < 1e-5


def test_resample_argument_errors(gpu_lib):
    api = gpu_lib
    lib = api.load_library()
    sino = torch.zeros(1, 8, 8, device="cuda")
    lino = torch.zeros(1, 4, 8, 8, device="cuda")
    p_s, p_l = sino.data_ptr(), lino.data_ptr()
    assert lib.fbp_resample_sinogram(p_s, p_l, 1, 6, 8, 8, None) == api.FBP_EINVAL   # N
    assert lib.fbp_resample_sinogram(p_s, p_l, 1, 8, 0, 8, None) == api.FBP_EINVAL   # angles
    assert lib.fbp_resample_sinogram(p_s, p_l, 1, 8, 8, 0, None) == api.FBP_EINVAL   # detector
    assert lib.fbp_resample_sinogram(None, p_l, 1, 8, 8, 8, None) == api.FBP_EINVAL
    assert lib.fbp_resample_sinogram(p_s, p_l + 4, 1, 8, 8, 8, None) == api.FBP_EINVAL
    assert lib.fbp_resample_sinogram(p_s, p_l, 0, 8, 8, 8, None) == api.FBP_OK
    assert lib.fbp_resample_sinogram(p_s, p_l, -1, 8, 8, 8, None) == api.FBP_EINVAL


def test_padded_grid_handles_objects_outside_the_disc(gpu_lib):
    """Ellipses filling the square (inside radius 0.65 N): on the N-shift linogram the
    projections of steep rows are longer than N and fold onto themselves (the cyclic shift
    axis holds objects inside 0.34 N only).  Reconstructed on the 2N grid and cropped, they
    come back about as well as in-disc objects do (measured on the CPU oracle: plain 0.75,
    padded 0.36 against the direct FBP; the rest is the order-4 filter's own error).  Measured
    against the FP64 direct FBP of the same sinogram; the composition is also held to the
    FP64 oracle of the same steps."""
    api = gpu_lib
    N, P, D, B = 128, 256, 256, 2
    ells = I.random_ellipses(N, 12, seed=31, disc=0.65, batch=B)
    sino = I.parallel_sinogram(ells, N, P, n_det=D, device="cuda", dtype=torch.float32)
    b4, a4, _ = api.fbp_fit_ramp_iir(4, 256, dc_zero=True)
    yard = O.fbp_direct_parallel(sino.cpu().double(), N)
    with api.fbp_plan(N, B, b4, a4) as plan, api.fbp_plan(2 * N, B, b4, a4) as plan2:
        plain = api.fbp_reconstruct_sinogram(plan, sino)
        padded = api.fbp_reconstruct_sinogram_padded(plan2, sino, N)
        torch.cuda.synchronize()
        e_plain = _rel(plain, yard)
        e_pad = _rel(padded, yard)
        assert e_pad < 0.6 * e_plain, (e_plain, e_pad)
        bc = np.array(plan2._b, np.float32).astype(np.float64)
        ac = np.array(plan2._a, np.float32).astype(np.float64)
    ref2 = O.fbp_fht(O.resample_sinogram(sino.cpu().double(), 2 * N), torch.tensor(bc[0]),
                     torch.tensor(ac[0]))
    o = N // 2
    assert _rel(padded, ref2[:, o:o + N, o:o + N]) < 1e-5
